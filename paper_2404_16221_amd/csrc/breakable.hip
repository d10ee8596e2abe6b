// Breakable integrals composited across regions (App. B.2, Properties 1-2).
//
// The family that the two properties generate from the transmittance, up to
// one level of nesting, over F per-sample channels f_c and P channel pairs
// (a_p, b_p), with w = T sigma the volume-rendering weight:
//   first order   Phi_c = int w f_c                      (Property 2 once)
//   second order  Psi_p = int w(u) a(u) [int_{v<u} w(v) b(v) dv] du
//                 (Property 1's product T * Phi_b, then Property 2 again;
//                 the distortion loss of the Examples is 2 (Psi_(m,1) -
//                 Psi_(1,m)) plus its within-sample term).
// Quadrature as in the colour path: piecewise-constant density and channels
// over each sample interval, w_i = T_i (1 - exp(-tau_i)), and
//   Phi_c = sum_i w_i f_ci,
//   Psi_p = sum_i w_i a_i sum_{j<i} w_j b_j + 1/2 sum_i w_i^2 a_i b_i
// (the last term is the exact within-interval part of the nested integral).
//
// A segment's tuple x = (tau, Phi[F], Psi[P]) folds front to back with
//   (x (+) y) = (tau_x + tau_y, Phi_x + T_x Phi_y,
//                Psi_x + T_x^2 Psi_y + T_x Phi_(a)y Phi_(b)x),
// which is what the proof of Property 2 does with its terms S_1 and S_2; (+)
// is associative with the zero tuple as identity.  The merge is one lane per
// ray; its backward records each segment's prefix transmittance and Phi_b in
// the segment's own gradient entries, then carries the suffix fold S in a
// reverse sweep and takes the Jacobian of P (+) x (+) S with respect to x.
//
// Segment kernels: one wave per segment, 64 samples per step, DPP scans
// for the optical depth, the prefix sums of w b_p (forward) and the prefix
// sums of w a_p and of w v (backward).  Per-sample suffix sums in the backward
// are a segment total from the forward tuple minus the inclusive prefix (Phi_a
// for sum_{j>i} w_j a_j, sum_c g_c Phi_c + 2 sum_p h_p Psi_p for sum_{j>i} w_j
// v_j), so their rounding error is absolute, about one float32 ulp of that
// total.
//
// Channel sources: loaded from a [n][F] array in the storage type, or the
// powers 1, m, m^2, ... of the sample midpoint, formed in the kernel (the
// depth moments; they carry no gradient).
#include <hip/hip_runtime.h>

#include "../../include/xl.h"
#include "internal.h"
#include "xl_device.hpp"

namespace xl {
namespace {

constexpr int kMaxCh = XL_BREAKABLE_MAX_CH;
constexpr int kMaxPairs = XL_BREAKABLE_MAX_PAIRS;
constexpr int kBrWaves = 4;
constexpr int kBrBlock = kBrWaves * kWave;
constexpr int kBrMergeBlock = 256;
constexpr int kXcdCount = 8;  // workgroups go to the 8 XCDs round robin

struct BrDev {
  const void* sigma;
  const void* ch;
  const float* t0;
  const float* t1;
  int F, P;
  int pa[kMaxPairs], pb[kMaxPairs];
};

// Wave scans on DPP (no LDS round trip): row shifts by 1, 2, 4, 8 inside each
// row of 16 lanes, then rows 1 and 3 add the last lane of the row below and
// rows 2-3 lane 31.  Lanes without a source, and disabled rows, read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp0(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                               ROW_MASK, 0xF, true));
}
__device__ __forceinline__ float incl_sum(float v) {
  v += dpp0<kRowShr1, 0xF>(v);
  v += dpp0<kRowShr2, 0xF>(v);
  v += dpp0<kRowShr4, 0xF>(v);
  v += dpp0<kRowShr8, 0xF>(v);
  v += dpp0<kRowBcast15, 0xA>(v);
  v += dpp0<kRowBcast31, 0xC>(v);
  return v;
}
// Exclusive prefix from an inclusive one (lane 0 gets 0).
__device__ __forceinline__ float excl_of(float incl) { return dpp0<kWaveShr1, 0xF>(incl); }
__device__ __forceinline__ float wave_total(float incl) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, incl), kWave - 1));
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

// f[idx] for a wave-uniform runtime index, without dynamic register indexing.
template <int FB>
__device__ __forceinline__ float pick(const float (&f)[FB], int idx) {
  float r = f[0];
#pragma unroll
  for (int c = 1; c < FB; ++c) r = idx == c ? f[c] : r;
  return r;
}

template <int DT>
__device__ __forceinline__ float load_one(const void* p, int64_t i) {
  if (DT == kF32) return static_cast<const float*>(p)[i];
  return to_f32<DT>(static_cast<const uint16_t*>(p)[i]);
}
template <int DT>
__device__ __forceinline__ void store_one(void* p, int64_t i, float v) {
  if (DT == kF32) static_cast<float*>(p)[i] = v;
  else static_cast<uint16_t*>(p)[i] = from_f32<DT>(v);
}

// Channels of sample i (zero past F; FB >= F is the kernel's channel bound).
template <int DT, int SRC, int FB>
__device__ __forceinline__ void channels(const BrDev& s, int64_t i, float m, float (&f)[FB]) {
  if (SRC == XL_CH_MIDPOINT_POWERS) {
    float p = 1.f;
#pragma unroll
    for (int c = 0; c < FB; ++c) {
      f[c] = c < s.F ? p : 0.f;
      p *= m;
    }
  } else {
#pragma unroll
    for (int c = 0; c < FB; ++c) f[c] = c < s.F ? load_one<DT>(s.ch, i * s.F + c) : 0.f;
  }
}

// Optical depth of the earlier steps of a segment, compensated (TwoSum).
struct DepthSum {
  float hi = 0.f, lo = 0.f;
  __device__ __forceinline__ void add(float x) {
    float e;
    hi = two_sum(hi, x, e);
    lo += e;
  }
  __device__ __forceinline__ float value() const { return hi + lo; }
};

// One sample of a step: its interval, optical depth and weight.
struct BrSample {
  bool in;
  float delta, m, od, e, T, w;
};

template <int DT>
__device__ __forceinline__ BrSample br_sample(const BrDev& s, int64_t i, bool in, float before,
                                              float& step_depth) {
  BrSample q;
  q.in = in;
  q.delta = 0.f;
  q.m = 0.f;
  q.od = 0.f;
  if (in) {
    const float t0 = s.t0[i], t1 = s.t1[i];
    q.delta = t1 - t0;
    q.m = 0.5f * (t0 + t1);
    q.od = load_one<DT>(s.sigma, i) * q.delta;
  }
  const float incl = incl_sum(q.od);
  q.e = exp_neg(q.od);
  q.T = exp_neg(before + (incl - q.od));
  q.w = q.T * one_minus_exp_neg(q.od, q.e);
  step_depth = wave_total(incl);
  return q;
}

template <int DT, int SRC, int FB>
__global__ __launch_bounds__(kBrBlock) void br_fwd_kernel(BrDev s, const int64_t* __restrict__ so,
                                                          int64_t n_seg, float* __restrict__ out) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kBrWaves + wave;
  if (k >= n_seg) return;
  const int64_t a = so[k], b = so[k + 1];
  float phi[FB], psi[kMaxPairs], wb_before[kMaxPairs];
#pragma unroll
  for (int c = 0; c < FB; ++c) phi[c] = 0.f;
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p) psi[p] = wb_before[p] = 0.f;
  DepthSum before;
  for (int64_t base = a; base < b; base += kWave) {
    const int64_t i = base + lane;
    float step;
    const BrSample q = br_sample<DT>(s, i, i < b, before.value(), step);
    float f[FB];
    if (q.in) channels<DT, SRC, FB>(s, i, q.m, f);
    else {
#pragma unroll
      for (int c = 0; c < FB; ++c) f[c] = 0.f;
    }
#pragma unroll
    for (int c = 0; c < FB; ++c) phi[c] = fmaf(q.w, f[c], phi[c]);
#pragma unroll
    for (int p = 0; p < kMaxPairs; ++p) {
      if (p < s.P) {
        const float av = pick(f, s.pa[p]), bv = pick(f, s.pb[p]);
        const float wb = q.w * bv;
        const float ib = incl_sum(wb);
        const float wa = q.w * av;
        psi[p] = fmaf(wa, wb_before[p] + excl_of(ib) + 0.5f * wb, psi[p]);
        wb_before[p] += wave_total(ib);
      }
    }
    before.add(step);
  }
  const int F = s.F, P = s.P;
  float mine = 0.f;  // lane c of the output row gets channel c's total
#pragma unroll
  for (int c = 0; c < FB; ++c) {
    if (c < F) {
      const float t = wave_sum(phi[c]);
      mine = lane == 1 + c ? t : mine;
    }
  }
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p) {
    if (p < P) {
      const float t = wave_sum(psi[p]);
      mine = lane == 1 + F + p ? t : mine;
    }
  }
  mine = lane == 0 ? before.value() : mine;
  if (lane < 1 + F + P) out[lane * n_seg + k] = mine;
}

template <int DT, int SRC, int FB>
__global__ __launch_bounds__(kBrBlock) void br_bwd_kernel(BrDev s, const int64_t* __restrict__ so,
                                                          int64_t n_seg,
                                                          const float* __restrict__ seg_out,
                                                          const float* __restrict__ gseg,
                                                          void* __restrict__ grad_sigma,
                                                          void* __restrict__ grad_ch, int accumulate) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kBrWaves + wave;
  if (k >= n_seg) return;
  const int64_t a = so[k], b = so[k + 1];
  const int F = s.F, P = s.P;
  const float g_tau = gseg[k];
  float g[FB], h[kMaxPairs], phi_a[kMaxPairs];
  float vtot = 0.f;  // sum over the segment of w_i v_i
#pragma unroll
  for (int c = 0; c < FB; ++c) {
    g[c] = c < F ? gseg[(1 + c) * n_seg + k] : 0.f;
    if (c < F) vtot = fmaf(g[c], seg_out[(1 + c) * n_seg + k], vtot);
  }
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p) {
    h[p] = p < P ? gseg[(1 + F + p) * n_seg + k] : 0.f;
    phi_a[p] = p < P ? seg_out[(1 + s.pa[p]) * n_seg + k] : 0.f;
    if (p < P) vtot = fmaf(2.f * h[p], seg_out[(1 + F + p) * n_seg + k], vtot);
  }
  DepthSum before;
  float wb_before[kMaxPairs], wa_before[kMaxPairs];
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p) wb_before[p] = wa_before[p] = 0.f;
  float vpre = 0.f;
  for (int64_t base = a; base < b; base += kWave) {
    const int64_t i = base + lane;
    float step;
    const BrSample q = br_sample<DT>(s, i, i < b, before.value(), step);
    float f[FB];
    if (q.in) channels<DT, SRC, FB>(s, i, q.m, f);
    else {
#pragma unroll
      for (int c = 0; c < FB; ++c) f[c] = 0.f;
    }
    float v = 0.f;
#pragma unroll
    for (int c = 0; c < FB; ++c) v = fmaf(g[c], f[c], v);
    float wb_lt[kMaxPairs], wa_gt[kMaxPairs], av[kMaxPairs], bv[kMaxPairs];
#pragma unroll
    for (int p = 0; p < kMaxPairs; ++p) {
      wb_lt[p] = wa_gt[p] = av[p] = bv[p] = 0.f;
      if (p < P) {
        av[p] = pick(f, s.pa[p]);
        bv[p] = pick(f, s.pb[p]);
        const float ib = incl_sum(q.w * bv[p]);
        const float ia = incl_sum(q.w * av[p]);
        wb_lt[p] = wb_before[p] + excl_of(ib);          // sum_{j<i} w_j b_j
        wa_gt[p] = phi_a[p] - (wa_before[p] + ia);            // sum_{j>i} w_j a_j
        wb_before[p] += wave_total(ib);
        wa_before[p] += wave_total(ia);
        // dPsi_p/dw_i
        const float U = fmaf(av[p], wb_lt[p], fmaf(bv[p], wa_gt[p], q.w * av[p] * bv[p]));
        v = fmaf(h[p], U, v);
      }
    }
    const float iu = incl_sum(q.w * v);
    const float v_gt = vtot - (vpre + iu);  // sum_{j>i} w_j v_j
    const float dtau = g_tau + q.T * q.e * v - v_gt;
    vpre += wave_total(iu);
    before.add(step);
    if (q.in) {
      float ds = q.delta * dtau;
      if (accumulate) ds += load_one<DT>(grad_sigma, i);
      store_one<DT>(grad_sigma, i, ds);
      if (SRC == XL_CH_LOADED) {
#pragma unroll
        for (int c = 0; c < FB; ++c) {
          if (c < F) {
            float df = q.w * g[c];
#pragma unroll
            for (int p = 0; p < kMaxPairs; ++p) {
              if (p < P) {
                if (s.pa[p] == c) df = fmaf(h[p], q.w * fmaf(0.5f * q.w, bv[p], wb_lt[p]), df);
                if (s.pb[p] == c) df = fmaf(h[p], q.w * fmaf(0.5f * q.w, av[p], wa_gt[p]), df);
              }
            }
            store_one<DT>(grad_ch, i * F + c, df);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- merge
__device__ __forceinline__ int64_t br_ray(int64_t n_rays) {
  const int64_t nblocks = (n_rays + kBrMergeBlock - 1) / kBrMergeBlock;
  const int64_t per = (nblocks + kXcdCount - 1) / kXcdCount;
  const int64_t bk = blockIdx.x;
  return ((bk % kXcdCount) * per + bk / kXcdCount) * kBrMergeBlock + threadIdx.x;
}

__device__ __forceinline__ void ray_range(const int64_t* __restrict__ ro, int64_t r, int64_t n_seg,
                                          int64_t& k0, int64_t& k1) {
  k0 = ro[r];
  k1 = ro[r + 1];
  k0 = k0 < 0 ? 0 : (k0 > n_seg ? n_seg : k0);
  k1 = k1 < k0 ? k0 : (k1 > n_seg ? n_seg : k1);
}

struct BrTup {
  float tau;
  float phi[kMaxCh];
  float psi[kMaxPairs];
};

__device__ __forceinline__ void load_tup(const float* __restrict__ x, int64_t n_seg, int64_t sg,
                                         int F, int P, BrTup& t) {
  t.tau = x[sg];
#pragma unroll
  for (int c = 0; c < kMaxCh; ++c) t.phi[c] = c < F ? x[(1 + c) * n_seg + sg] : 0.f;
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p) t.psi[p] = p < P ? x[(1 + F + p) * n_seg + sg] : 0.f;
}

__global__ __launch_bounds__(kBrMergeBlock) void br_merge_fwd_kernel(
    BrDev s, const float* __restrict__ seg_out, int64_t n_seg, const int64_t* __restrict__ ro,
    const int64_t* __restrict__ ids, int64_t n_rays, float* __restrict__ out) {
  const int64_t r = br_ray(n_rays);
  if (r >= n_rays) return;
  const int F = s.F, P = s.P;
  int64_t k0, k1;
  ray_range(ro, r, n_seg, k0, k1);
  DepthSum tau;
  float T = 1.f, phi[kMaxCh], psi[kMaxPairs], G[kMaxPairs];
#pragma unroll
  for (int c = 0; c < kMaxCh; ++c) phi[c] = 0.f;
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p) psi[p] = G[p] = 0.f;
  for (int64_t q = k0; q < k1; ++q) {
    const int64_t sg = ids[q];
    if (sg < 0 || sg >= n_seg) continue;
    BrTup x;
    load_tup(seg_out, n_seg, sg, F, P, x);
#pragma unroll
    for (int p = 0; p < kMaxPairs; ++p) {
      if (p < P) {
        // the pair's channels, read again rather than selected from x
        const float xa = seg_out[(1 + s.pa[p]) * n_seg + sg];
        const float xb = seg_out[(1 + s.pb[p]) * n_seg + sg];
        psi[p] = fmaf(T * T, x.psi[p], fmaf(T * xa, G[p], psi[p]));
        G[p] = fmaf(T, xb, G[p]);
      }
    }
#pragma unroll
    for (int c = 0; c < kMaxCh; ++c) phi[c] = fmaf(T, x.phi[c], phi[c]);
    tau.add(x.tau);
    T = exp_neg(tau.value());
  }
  out[r] = T;
#pragma unroll
  for (int c = 0; c < kMaxCh; ++c)
    if (c < F) out[(1 + c) * n_rays + r] = phi[c];
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p)
    if (p < P) out[(1 + F + p) * n_rays + r] = psi[p];
}

__global__ __launch_bounds__(kBrMergeBlock) void br_merge_bwd_kernel(
    BrDev s, const float* __restrict__ seg_out, int64_t n_seg, const int64_t* __restrict__ ro,
    const int64_t* __restrict__ ids, int64_t n_rays, const float* __restrict__ gray,
    float* __restrict__ gseg) {
  const int64_t r = br_ray(n_rays);
  if (r >= n_rays) return;
  const int F = s.F, P = s.P;
  int64_t k0, k1;
  ray_range(ro, r, n_seg, k0, k1);
  const float gT = gray[r];
  float g[kMaxCh], h[kMaxPairs];
#pragma unroll
  for (int c = 0; c < kMaxCh; ++c) g[c] = c < F ? gray[(1 + c) * n_rays + r] : 0.f;
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p) h[p] = p < P ? gray[(1 + F + p) * n_rays + r] : 0.f;
  // Forward sweep: the prefix transmittance and Phi_b of every segment,
  // parked in the segment's tau and Psi gradient entries.
  {
    DepthSum tau;
    float T = 1.f, G[kMaxPairs];
#pragma unroll
    for (int p = 0; p < kMaxPairs; ++p) G[p] = 0.f;
    for (int64_t q = k0; q < k1; ++q) {
      const int64_t sg = ids[q];
      if (sg < 0 || sg >= n_seg) continue;
      gseg[sg] = T;
#pragma unroll
      for (int p = 0; p < kMaxPairs; ++p) {
        if (p < P) {
          gseg[(1 + F + p) * n_seg + sg] = G[p];
          G[p] = fmaf(T, seg_out[(1 + s.pb[p]) * n_seg + sg], G[p]);
        }
      }
      tau.add(seg_out[sg]);
      T = exp_neg(tau.value());
    }
  }
  // Reverse sweep with the suffix fold S (Sa: its Phi_a of every pair).
  BrTup S;
  S.tau = 0.f;
  float Sa[kMaxPairs];
#pragma unroll
  for (int c = 0; c < kMaxCh; ++c) S.phi[c] = 0.f;
#pragma unroll
  for (int p = 0; p < kMaxPairs; ++p) S.psi[p] = Sa[p] = 0.f;
  DepthSum stau;
  for (int64_t q = k1 - 1; q >= k0; --q) {
    const int64_t sg = ids[q];
    if (sg < 0 || sg >= n_seg) continue;
    BrTup x;
    load_tup(seg_out, n_seg, sg, F, P, x);
    const float PT = gseg[sg];
    const float xT = exp_neg(x.tau), ST = exp_neg(stau.value());
    float dxT = PT * gT * ST;
#pragma unroll
    for (int c = 0; c < kMaxCh; ++c) dxT = fmaf(g[c] * PT, S.phi[c], dxT);
    float dphi[kMaxCh], xa[kMaxPairs], xb[kMaxPairs];
#pragma unroll
    for (int c = 0; c < kMaxCh; ++c) dphi[c] = g[c] * PT;
#pragma unroll
    for (int p = 0; p < kMaxPairs; ++p) {
      xa[p] = xb[p] = 0.f;
      if (p < P) {
        const float PFb = gseg[(1 + F + p) * n_seg + sg];
        xa[p] = seg_out[(1 + s.pa[p]) * n_seg + sg];
        xb[p] = seg_out[(1 + s.pb[p]) * n_seg + sg];
        dxT = fmaf(h[p] * PT * PT, fmaf(2.f * xT, S.psi[p], Sa[p] * xb[p]), dxT);
        dxT = fmaf(h[p] * PT * Sa[p], PFb, dxT);
#pragma unroll
        for (int c = 0; c < kMaxCh; ++c) {
          if (s.pa[p] == c) dphi[c] = fmaf(h[p] * PT, PFb, dphi[c]);
          if (s.pb[p] == c) dphi[c] = fmaf(h[p] * PT * PT * xT, Sa[p], dphi[c]);
        }
        gseg[(1 + F + p) * n_seg + sg] = h[p] * PT * PT;
      }
    }
    gseg[sg] = -xT * dxT;
#pragma unroll
    for (int c = 0; c < kMaxCh; ++c)
      if (c < F) gseg[(1 + c) * n_seg + sg] = dphi[c];
    // S <- x (+) S
#pragma unroll
    for (int p = 0; p < kMaxPairs; ++p) {
      S.psi[p] = fmaf(xT * Sa[p], xb[p], fmaf(xT * xT, S.psi[p], x.psi[p]));
      Sa[p] = fmaf(xT, Sa[p], xa[p]);
    }
#pragma unroll
    for (int c = 0; c < kMaxCh; ++c) S.phi[c] = fmaf(xT, S.phi[c], x.phi[c]);
    stau.add(x.tau);
  }
}

BrDev br_dev(const xl_breakable* d) {
  BrDev s;
  s.sigma = d->sigma;
  s.ch = d->ch;
  s.t0 = d->t_start;
  s.t1 = d->t_end;
  s.F = d->n_ch;
  s.P = d->n_pairs;
  for (int p = 0; p < kMaxPairs; ++p) {
    s.pa[p] = p < d->n_pairs ? d->pair_a[p] : 0;
    s.pb[p] = p < d->n_pairs ? d->pair_b[p] : 0;
  }
  return s;
}

// Channel loops run to 4 for up to four channels, else to kMaxCh.
template <int DT, int SRC>
void fwd_launch(const BrDev& s, const int64_t* so, int64_t n_seg, float* out, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n_seg + kBrWaves - 1) / kBrWaves)), block(kBrBlock);
  if (s.F <= 4)
    hipLaunchKernelGGL((br_fwd_kernel<DT, SRC, 4>), grid, block, 0, st, s, so, n_seg, out);
  else
    hipLaunchKernelGGL((br_fwd_kernel<DT, SRC, kMaxCh>), grid, block, 0, st, s, so, n_seg, out);
}

template <int DT, int SRC>
void bwd_launch(const BrDev& s, const int64_t* so, int64_t n_seg, const float* seg_out,
                const float* gseg, void* gs, void* gc, int acc, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n_seg + kBrWaves - 1) / kBrWaves)), block(kBrBlock);
  if (s.F <= 4)
    hipLaunchKernelGGL((br_bwd_kernel<DT, SRC, 4>), grid, block, 0, st, s, so, n_seg, seg_out, gseg,
                       gs, gc, acc);
  else
    hipLaunchKernelGGL((br_bwd_kernel<DT, SRC, kMaxCh>), grid, block, 0, st, s, so, n_seg, seg_out,
                       gseg, gs, gc, acc);
}

unsigned br_merge_grid(int64_t n_rays) {
  const int64_t nblocks = (n_rays + kBrMergeBlock - 1) / kBrMergeBlock;
  return static_cast<unsigned>((nblocks + kXcdCount - 1) / kXcdCount * kXcdCount);
}

}  // namespace

hipError_t launch_breakable_fwd(const xl_breakable* d, const int64_t* so, int64_t n_seg,
                                float* seg_out, hipStream_t st) {
  if (n_seg <= 0) return hipSuccess;
  const BrDev s = br_dev(d);
  const bool mp = d->source == XL_CH_MIDPOINT_POWERS;
  switch (d->dtype) {
    case kF32: mp ? fwd_launch<kF32, XL_CH_MIDPOINT_POWERS>(s, so, n_seg, seg_out, st)
                  : fwd_launch<kF32, XL_CH_LOADED>(s, so, n_seg, seg_out, st); break;
    case kBF16: mp ? fwd_launch<kBF16, XL_CH_MIDPOINT_POWERS>(s, so, n_seg, seg_out, st)
                   : fwd_launch<kBF16, XL_CH_LOADED>(s, so, n_seg, seg_out, st); break;
    default: mp ? fwd_launch<kF16, XL_CH_MIDPOINT_POWERS>(s, so, n_seg, seg_out, st)
                : fwd_launch<kF16, XL_CH_LOADED>(s, so, n_seg, seg_out, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_breakable_bwd(const xl_breakable* d, const int64_t* so, int64_t n_seg,
                                const float* seg_out, const float* grad_seg, void* grad_sigma,
                                void* grad_ch, int accumulate, hipStream_t st) {
  if (n_seg <= 0) return hipSuccess;
  const BrDev s = br_dev(d);
  const bool mp = d->source == XL_CH_MIDPOINT_POWERS;
  switch (d->dtype) {
    case kF32: mp ? bwd_launch<kF32, XL_CH_MIDPOINT_POWERS>(s, so, n_seg, seg_out, grad_seg, grad_sigma, grad_ch, accumulate, st)
                  : bwd_launch<kF32, XL_CH_LOADED>(s, so, n_seg, seg_out, grad_seg, grad_sigma, grad_ch, accumulate, st); break;
    case kBF16: mp ? bwd_launch<kBF16, XL_CH_MIDPOINT_POWERS>(s, so, n_seg, seg_out, grad_seg, grad_sigma, grad_ch, accumulate, st)
                   : bwd_launch<kBF16, XL_CH_LOADED>(s, so, n_seg, seg_out, grad_seg, grad_sigma, grad_ch, accumulate, st); break;
    default: mp ? bwd_launch<kF16, XL_CH_MIDPOINT_POWERS>(s, so, n_seg, seg_out, grad_seg, grad_sigma, grad_ch, accumulate, st)
                : bwd_launch<kF16, XL_CH_LOADED>(s, so, n_seg, seg_out, grad_seg, grad_sigma, grad_ch, accumulate, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_breakable_merge(const xl_breakable* d, const float* seg_out, int64_t n_seg,
                                  const int64_t* ro, const int64_t* ids, int64_t n_rays,
                                  float* ray_out, hipStream_t st) {
  if (n_rays <= 0) return hipSuccess;
  const BrDev s = br_dev(d);
  hipLaunchKernelGGL(br_merge_fwd_kernel, dim3(br_merge_grid(n_rays)), dim3(kBrMergeBlock), 0, st, s,
                     seg_out, n_seg, ro, ids, n_rays, ray_out);
  return hipGetLastError();
}

hipError_t launch_breakable_merge_bwd(const xl_breakable* d, const float* seg_out, int64_t n_seg,
                                      const int64_t* ro, const int64_t* ids, int64_t n_rays,
                                      const float* grad_ray, float* grad_seg, hipStream_t st) {
  if (n_rays <= 0) return hipSuccess;
  const BrDev s = br_dev(d);
  hipLaunchKernelGGL(br_merge_bwd_kernel, dim3(br_merge_grid(n_rays)), dim3(kBrMergeBlock), 0, st, s,
                     seg_out, n_seg, ro, ids, n_rays, grad_ray, grad_seg);
  return hipGetLastError();
}

}  // namespace xl
