// Feature channels composited across regions (App. B.2).  Breakable integrals
// are closed under integration against a breakable factor (Property 2); with
// the transmittance as that factor, any per-sample feature vector f_i rendered
// with the volume-rendering weights splits over segments like colour:
//   segment   Phi_k = sum_i w_i f_i,  w_i = T_i (1 - exp(-tau_i)), T from 1,
//   ray       Phi   = sum_k exp(-sum_{j<k} tau_j) Phi_k, front to back.
// Backward, per sample of segment k with g = dl/dPhi_k and p_i = g . f_i:
//   dl/dtau_i = g_tau_k + T_{i+1} p_i - sum_{j>i} w_j p_j,  dl/df_i = w_i g,
// the suffix taken as g . Phi_k minus the inclusive prefix; g_tau_k is the
// merge's gradient through the transmittance of later segments.
//
// One wave per segment walks its samples 64 at a time (one per lane) with a
// wave scan of the optical depths; a lane loads its sample's feature row as
// 16-byte vectors (rows are contiguous across the wave) and keeps partial
// sums, reduced once per segment.  F is 4, 8, 16 or 32.
#include <hip/hip_runtime.h>

#include "../../include/xl.h"
#include "internal.h"
#include "xl_device.hpp"

namespace xl {
namespace {

constexpr int kFeatWaves = 4;
constexpr int kFeatBlock = kFeatWaves * kWave;

__device__ __forceinline__ float wave_incl_sum(float v, int lane) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const float y = __shfl_up(v, d);
    if (lane >= d) v += y;
  }
  return v;
}

template <int DT>
__device__ __forceinline__ float load_scalar(const void* p, int64_t i) {
  if (DT == kF32) return static_cast<const float*>(p)[i];
  return to_f32<DT>(static_cast<const uint16_t*>(p)[i]);
}

template <int DT>
__device__ __forceinline__ void store_scalar(void* p, int64_t i, float v) {
  if (DT == kF32) static_cast<float*>(p)[i] = v;
  else static_cast<uint16_t*>(p)[i] = from_f32<DT>(v);
}

// Row i of a [n][F] feature array, as F floats.
template <int DT, int F>
__device__ __forceinline__ void load_row(const void* p, int64_t i, float (&f)[F]) {
  if (DT == kF32) {
    const float4* q = reinterpret_cast<const float4*>(static_cast<const float*>(p) + i * F);
#pragma unroll
    for (int v = 0; v < F / 4; ++v) {
      const float4 x = q[v];
      f[4 * v] = x.x; f[4 * v + 1] = x.y; f[4 * v + 2] = x.z; f[4 * v + 3] = x.w;
    }
  } else if (F == 4) {
    const uint2 x = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(p) + i * F);
    const uint32_t w[2] = {x.x, x.y};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      f[2 * c] = to_f32<DT>(static_cast<uint16_t>(w[c] & 0xFFFFu));
      f[2 * c + 1] = to_f32<DT>(static_cast<uint16_t>(w[c] >> 16));
    }
  } else {
    const uint4* q = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(p) + i * F);
#pragma unroll
    for (int v = 0; v < F / 8; ++v) {
      const uint4 x = q[v];
      const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        f[8 * v + 2 * c] = to_f32<DT>(static_cast<uint16_t>(w[c] & 0xFFFFu));
        f[8 * v + 2 * c + 1] = to_f32<DT>(static_cast<uint16_t>(w[c] >> 16));
      }
    }
  }
}

template <int DT, int F>
__device__ __forceinline__ void store_row(void* p, int64_t i, const float (&f)[F]) {
  if (DT == kF32) {
    float4* q = reinterpret_cast<float4*>(static_cast<float*>(p) + i * F);
#pragma unroll
    for (int v = 0; v < F / 4; ++v) q[v] = make_float4(f[4 * v], f[4 * v + 1], f[4 * v + 2], f[4 * v + 3]);
  } else if (F == 4) {
    *reinterpret_cast<uint2*>(static_cast<uint16_t*>(p) + i * F) =
        make_uint2(pack2<DT>(f[0], f[1]), pack2<DT>(f[2], f[3]));
  } else {
    uint4* q = reinterpret_cast<uint4*>(static_cast<uint16_t*>(p) + i * F);
#pragma unroll
    for (int v = 0; v < F / 8; ++v)
      q[v] = make_uint4(pack2<DT>(f[8 * v], f[8 * v + 1]), pack2<DT>(f[8 * v + 2], f[8 * v + 3]),
                        pack2<DT>(f[8 * v + 4], f[8 * v + 5]), pack2<DT>(f[8 * v + 6], f[8 * v + 7]));
  }
}

struct FeatDev {
  const void* sigma;
  const void* feat;
  const float* t0;
  const float* t1;
};

template <int DT, int F>
__global__ __launch_bounds__(kFeatBlock) void feat_fwd_kernel(FeatDev s, const int64_t* __restrict__ seg_offsets,
                                                              int64_t n_seg, float* __restrict__ phi,
                                                              float* __restrict__ tau_seg) {
  __shared__ float red[kFeatWaves][kWave * (F + 1)];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kFeatWaves + wave;
  if (k >= n_seg) return;
  const int64_t a = seg_offsets[k], b = seg_offsets[k + 1];
  float acc[F];
#pragma unroll
  for (int c = 0; c < F; ++c) acc[c] = 0.f;
  float before = 0.f;  // optical depth of the segment's earlier chunks
  for (int64_t base = a; base < b; base += kWave) {
    const int64_t i = base + lane;
    const bool in = i < b;
    float od = 0.f;
    float f[F];
    if (in) {
      od = load_scalar<DT>(s.sigma, i) * (s.t1[i] - s.t0[i]);
      load_row<DT, F>(s.feat, i, f);
    } else {
#pragma unroll
      for (int c = 0; c < F; ++c) f[c] = 0.f;
    }
    const float incl = wave_incl_sum(od, lane);
    const float e = exp_neg(od);
    const float w = exp_neg(before + incl - od) * one_minus_exp_neg(od, e);
#pragma unroll
    for (int c = 0; c < F; ++c) acc[c] = fmaf(w, f[c], acc[c]);
    before += __shfl(incl, kWave - 1);
  }
  // Channel sums through a transpose in the wave's own LDS rows (a wave's
  // LDS operations run in order): lane (part, ch) adds F rows of channel ch,
  // then log2(64 / F) shuffles join the parts -- instead of 6 F shuffles.
  float* row = &red[wave][lane * (F + 1)];
#pragma unroll
  for (int c = 0; c < F; ++c) row[c] = acc[c];
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const int ch = lane % F, part = lane / F;
  float t = 0.f;
#pragma unroll
  for (int j = 0; j < F; ++j) t += red[wave][(part * F + j) * (F + 1) + ch];
#pragma unroll
  for (int d = F; d < kWave; d <<= 1) t += __shfl_xor(t, d);
  if (lane < F) phi[lane * n_seg + k] = t;
  if (tau_seg && lane == 0) tau_seg[k] = before;
}

// A ray's id range, clamped to the id array [0, n_seg) (a malformed offset
// array gives empty or shortened rays, never reads outside it).
__device__ __forceinline__ void ray_range(const int64_t* __restrict__ ro, int64_t r, int64_t n_seg,
                                          int64_t& q0, int64_t& q1) {
  q0 = ro[r];
  q1 = ro[r + 1];
  q0 = q0 < 0 ? 0 : (q0 > n_seg ? n_seg : q0);
  q1 = q1 < q0 ? q0 : (q1 > n_seg ? n_seg : q1);
}

// Running optical depth in front of a segment as a compensated pair (TwoSum),
// so that a ray's log-transmittance keeps its relative accuracy however many
// segments it crosses.
struct DepthSum {
  float hi = 0.f, lo = 0.f;
  __device__ __forceinline__ void add(float x) {
    float e;
    hi = two_sum(hi, x, e);
    lo += e;
  }
  __device__ __forceinline__ float value() const { return hi + lo; }
};

template <int F>
__global__ void feat_merge_fwd_kernel(const float* __restrict__ tau_seg, const float* __restrict__ phi,
                                      int64_t n_seg, const int64_t* __restrict__ ray_offsets,
                                      const int64_t* __restrict__ seg_ids, int64_t n_rays,
                                      float* __restrict__ out) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  float acc[F];
#pragma unroll
  for (int c = 0; c < F; ++c) acc[c] = 0.f;
  int64_t q0, q1;
  ray_range(ray_offsets, r, n_seg, q0, q1);
  DepthSum before;
  for (int64_t q = q0; q < q1; ++q) {
    const int64_t sg = seg_ids[q];
    if (sg < 0 || sg >= n_seg) continue;  // invalid ids are identities
    const float T = exp_neg(before.value());
#pragma unroll
    for (int c = 0; c < F; ++c) acc[c] = fmaf(T, phi[c * n_seg + sg], acc[c]);
    before.add(tau_seg[sg]);
  }
#pragma unroll
  for (int c = 0; c < F; ++c) out[c * n_rays + r] = acc[c];
}

// dl/dPhi_k = T_{<k} g and dl/dtau_k = -sum_{k' > k} T_{<k'} (g . Phi_k'): a
// forward pass stores each segment's preceding depth in grad_tau, a reverse
// pass turns it into the gradient.
template <int F>
__global__ void feat_merge_bwd_kernel(const float* __restrict__ tau_seg, const float* __restrict__ phi,
                                      int64_t n_seg, const int64_t* __restrict__ ray_offsets,
                                      const int64_t* __restrict__ seg_ids, int64_t n_rays,
                                      const float* __restrict__ grad_ray, float* __restrict__ gphi,
                                      float* __restrict__ gtau) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  float g[F];
#pragma unroll
  for (int c = 0; c < F; ++c) g[c] = grad_ray[c * n_rays + r];
  int64_t q0, q1;
  ray_range(ray_offsets, r, n_seg, q0, q1);
  DepthSum before;
  for (int64_t q = q0; q < q1; ++q) {
    const int64_t sg = seg_ids[q];
    if (sg < 0 || sg >= n_seg) continue;
    const float d = before.value();
    const float T = exp_neg(d);
#pragma unroll
    for (int c = 0; c < F; ++c) gphi[c * n_seg + sg] = T * g[c];
    gtau[sg] = d;
    before.add(tau_seg[sg]);
  }
  float later = 0.f;  // sum over later segments of T_{<k'} (g . Phi_k')
  for (int64_t q = q1 - 1; q >= q0; --q) {
    const int64_t sg = seg_ids[q];
    if (sg < 0 || sg >= n_seg) continue;
    const float T = exp_neg(gtau[sg]);
    float dot = 0.f;
#pragma unroll
    for (int c = 0; c < F; ++c) dot = fmaf(g[c], phi[c * n_seg + sg], dot);
    gtau[sg] = -later;
    later = fmaf(T, dot, later);
  }
}

template <int DT, int F>
__global__ __launch_bounds__(kFeatBlock) void feat_bwd_kernel(FeatDev s, const int64_t* __restrict__ seg_offsets,
                                                              int64_t n_seg, const float* __restrict__ phi,
                                                              const float* __restrict__ gphi,
                                                              const float* __restrict__ gtau,
                                                              void* __restrict__ grad_sigma,
                                                              void* __restrict__ grad_feat, int accumulate) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kFeatWaves + wave;
  if (k >= n_seg) return;
  const int64_t a = seg_offsets[k], b = seg_offsets[k + 1];
  float g[F];
  float gdot = 0.f;  // g . Phi_k = sum over the segment of w_j p_j
#pragma unroll
  for (int c = 0; c < F; ++c) {
    g[c] = gphi[c * n_seg + k];
    gdot = fmaf(g[c], phi[c * n_seg + k], gdot);
  }
  const float gt = gtau ? gtau[k] : 0.f;
  float before = 0.f, upre = 0.f;  // depth and sum of w p over earlier chunks
  for (int64_t base = a; base < b; base += kWave) {
    const int64_t i = base + lane;
    const bool in = i < b;
    float od = 0.f, delta = 0.f;
    float f[F];
    if (in) {
      delta = s.t1[i] - s.t0[i];
      od = load_scalar<DT>(s.sigma, i) * delta;
      load_row<DT, F>(s.feat, i, f);
    } else {
#pragma unroll
      for (int c = 0; c < F; ++c) f[c] = 0.f;
    }
    const float incl = wave_incl_sum(od, lane);
    const float e = exp_neg(od);
    const float T = exp_neg(before + incl - od);
    const float w = T * one_minus_exp_neg(od, e);
    float p = 0.f;
#pragma unroll
    for (int c = 0; c < F; ++c) p = fmaf(g[c], f[c], p);
    const float u = w * p;
    const float uincl = wave_incl_sum(u, lane);
    const float suffix = gdot - (upre + uincl);  // sum_{j > i} w_j p_j
    const float dtau = gt + T * e * p - suffix;
    if (in) {
      float ds = delta * dtau;
      if (accumulate) ds += load_scalar<DT>(grad_sigma, i);
      store_scalar<DT>(grad_sigma, i, ds);
      float df[F];
#pragma unroll
      for (int c = 0; c < F; ++c) df[c] = w * g[c];
      store_row<DT, F>(grad_feat, i, df);
    }
    before += __shfl(incl, kWave - 1);
    upre += __shfl(uincl, kWave - 1);
  }
}

template <int DT>
hipError_t fwd_dt(const FeatDev& s, int F, const int64_t* so, int64_t n_seg, float* phi, float* tau,
                  hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n_seg + kFeatWaves - 1) / kFeatWaves)), block(kFeatBlock);
  switch (F) {
    case 4: hipLaunchKernelGGL((feat_fwd_kernel<DT, 4>), grid, block, 0, st, s, so, n_seg, phi, tau); break;
    case 8: hipLaunchKernelGGL((feat_fwd_kernel<DT, 8>), grid, block, 0, st, s, so, n_seg, phi, tau); break;
    case 16: hipLaunchKernelGGL((feat_fwd_kernel<DT, 16>), grid, block, 0, st, s, so, n_seg, phi, tau); break;
    default: hipLaunchKernelGGL((feat_fwd_kernel<DT, 32>), grid, block, 0, st, s, so, n_seg, phi, tau); break;
  }
  return hipGetLastError();
}

template <int DT>
hipError_t bwd_dt(const FeatDev& s, int F, const int64_t* so, int64_t n_seg, const float* phi,
                  const float* gphi, const float* gtau, void* gs, void* gf, int acc, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((n_seg + kFeatWaves - 1) / kFeatWaves)), block(kFeatBlock);
  switch (F) {
    case 4: hipLaunchKernelGGL((feat_bwd_kernel<DT, 4>), grid, block, 0, st, s, so, n_seg, phi, gphi, gtau, gs, gf, acc); break;
    case 8: hipLaunchKernelGGL((feat_bwd_kernel<DT, 8>), grid, block, 0, st, s, so, n_seg, phi, gphi, gtau, gs, gf, acc); break;
    case 16: hipLaunchKernelGGL((feat_bwd_kernel<DT, 16>), grid, block, 0, st, s, so, n_seg, phi, gphi, gtau, gs, gf, acc); break;
    default: hipLaunchKernelGGL((feat_bwd_kernel<DT, 32>), grid, block, 0, st, s, so, n_seg, phi, gphi, gtau, gs, gf, acc); break;
  }
  return hipGetLastError();
}

FeatDev feat_dev(const xl_features* f) {
  FeatDev s;
  s.sigma = f->sigma;
  s.feat = f->feat;
  s.t0 = f->t_start;
  s.t1 = f->t_end;
  return s;
}

}  // namespace

hipError_t launch_features_fwd(const xl_features* f, const int64_t* seg_offsets, int64_t n_seg,
                               float* phi_seg, float* tau_seg, hipStream_t st) {
  if (n_seg <= 0) return hipSuccess;
  const FeatDev s = feat_dev(f);
  switch (f->dtype) {
    case kF32: return fwd_dt<kF32>(s, f->n_feat, seg_offsets, n_seg, phi_seg, tau_seg, st);
    case kBF16: return fwd_dt<kBF16>(s, f->n_feat, seg_offsets, n_seg, phi_seg, tau_seg, st);
    default: return fwd_dt<kF16>(s, f->n_feat, seg_offsets, n_seg, phi_seg, tau_seg, st);
  }
}

hipError_t launch_features_bwd(const xl_features* f, const int64_t* seg_offsets, int64_t n_seg,
                               const float* phi_seg, const float* grad_phi_seg, const float* grad_tau_seg,
                               void* grad_sigma, void* grad_feat, int accumulate, hipStream_t st) {
  if (n_seg <= 0) return hipSuccess;
  const FeatDev s = feat_dev(f);
  switch (f->dtype) {
    case kF32: return bwd_dt<kF32>(s, f->n_feat, seg_offsets, n_seg, phi_seg, grad_phi_seg, grad_tau_seg,
                                   grad_sigma, grad_feat, accumulate, st);
    case kBF16: return bwd_dt<kBF16>(s, f->n_feat, seg_offsets, n_seg, phi_seg, grad_phi_seg, grad_tau_seg,
                                     grad_sigma, grad_feat, accumulate, st);
    default: return bwd_dt<kF16>(s, f->n_feat, seg_offsets, n_seg, phi_seg, grad_phi_seg, grad_tau_seg,
                                 grad_sigma, grad_feat, accumulate, st);
  }
}

hipError_t launch_features_merge(const float* tau_seg, const float* phi_seg, int F, int64_t n_seg,
                                 const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                                 float* phi_ray, hipStream_t st) {
  if (n_rays <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((n_rays + 255) / 256)), block(256);
  switch (F) {
    case 4: hipLaunchKernelGGL(feat_merge_fwd_kernel<4>, grid, block, 0, st, tau_seg, phi_seg, n_seg, ray_offsets, seg_ids, n_rays, phi_ray); break;
    case 8: hipLaunchKernelGGL(feat_merge_fwd_kernel<8>, grid, block, 0, st, tau_seg, phi_seg, n_seg, ray_offsets, seg_ids, n_rays, phi_ray); break;
    case 16: hipLaunchKernelGGL(feat_merge_fwd_kernel<16>, grid, block, 0, st, tau_seg, phi_seg, n_seg, ray_offsets, seg_ids, n_rays, phi_ray); break;
    default: hipLaunchKernelGGL(feat_merge_fwd_kernel<32>, grid, block, 0, st, tau_seg, phi_seg, n_seg, ray_offsets, seg_ids, n_rays, phi_ray); break;
  }
  return hipGetLastError();
}

hipError_t launch_features_merge_bwd(const float* tau_seg, const float* phi_seg, int F, int64_t n_seg,
                                     const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                                     const float* grad_ray, float* grad_phi_seg, float* grad_tau_seg,
                                     hipStream_t st) {
  if (n_rays <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((n_rays + 255) / 256)), block(256);
  switch (F) {
    case 4: hipLaunchKernelGGL(feat_merge_bwd_kernel<4>, grid, block, 0, st, tau_seg, phi_seg, n_seg, ray_offsets, seg_ids, n_rays, grad_ray, grad_phi_seg, grad_tau_seg); break;
    case 8: hipLaunchKernelGGL(feat_merge_bwd_kernel<8>, grid, block, 0, st, tau_seg, phi_seg, n_seg, ray_offsets, seg_ids, n_rays, grad_ray, grad_phi_seg, grad_tau_seg); break;
    case 16: hipLaunchKernelGGL(feat_merge_bwd_kernel<16>, grid, block, 0, st, tau_seg, phi_seg, n_seg, ray_offsets, seg_ids, n_rays, grad_ray, grad_phi_seg, grad_tau_seg); break;
    default: hipLaunchKernelGGL(feat_merge_bwd_kernel<32>, grid, block, 0, st, tau_seg, phi_seg, n_seg, ray_offsets, seg_ids, n_rays, grad_ray, grad_phi_seg, grad_tau_seg); break;
  }
  return hipGetLastError();
}

}  // namespace xl
