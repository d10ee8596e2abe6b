// Merge of segment tuples in ray order (Sec. 4.3, Eq. 3-8; App. A.2, Alg. 1-2).
//
// One lane per ray folds the ray's segments front to back.  The transmittance
// in front of segment k is the exclusive product of the segment
// transmittances (Eq. 4), formed as exp(-sum_{j<k} tau_j); the distortion
// loss gains 2 T_{<k} S_k + T_{<k}^2 L_k with S_k = D_k A_{<k} - A_k D_{<k}
// (Eq. 7-8).  With XL_MERGE_FP64 the running sums and products are float64.
//
// The backward gives each segment the gradient of the merged tuple with
// respect to its own tuple only (the per-region differentiation rule of Sec.
// 4.2 and App. A.2): for segment k with exclusive prefix fold P and suffix fold
// S, the merged tuple is P (+) x_k (+) S, and the chain rule through the two
// (+) operations gives the per-component gradients below.  Rays with up to
// kCached segments hold their tuples and suffix folds in registers; longer rays
// compute the suffix folds by a reverse sweep and park them in grad_seg, which
// the forward sweep then overwrites with the gradients.
#include "internal.h"
#include "xl_device.hpp"

namespace xl {

template <typename R>
__device__ __forceinline__ R exp_neg_t(R x);
template <>
__device__ __forceinline__ float exp_neg_t<float>(float x) { return exp_neg(x); }  // as in the segment kernels
template <>
__device__ __forceinline__ double exp_neg_t<double>(double x) { return exp(-x); }

template <typename R>
struct Tup {
  R tau, cr, cg, cb, A, D, L;
  R tlo;  // compensation of tau (the exact optical depth is tau + tlo)
};

// Compensated accumulation of optical depths (Knuth's TwoSum on the high parts).
template <typename R>
__device__ __forceinline__ void add_tau_t(R& tau, R& tlo, R hi, R lo) {
  const R s = tau + hi;
  const R bb = s - tau;
  tlo += ((tau - (s - bb)) + (hi - bb)) + lo;
  tau = s;
}

template <typename R>
__device__ __forceinline__ Tup<R> load_tup(const float* __restrict__ p, int64_t n_seg, int64_t s) {
  Tup<R> x;
  x.tau = p[s]; x.cr = p[n_seg + s]; x.cg = p[2 * n_seg + s]; x.cb = p[3 * n_seg + s];
  x.A = p[4 * n_seg + s]; x.D = p[5 * n_seg + s]; x.L = p[6 * n_seg + s];
  x.tlo = 0;
  return x;
}

// x in front of y, with T_x = exp(-x.tau).
template <typename R>
__device__ __forceinline__ Tup<R> fold(const Tup<R>& x, R Tx, const Tup<R>& y) {
  Tup<R> r;
  r.tau = x.tau; r.tlo = x.tlo;
  add_tau_t<R>(r.tau, r.tlo, y.tau, y.tlo);
  r.cr = x.cr + Tx * y.cr; r.cg = x.cg + Tx * y.cg; r.cb = x.cb + Tx * y.cb;
  r.A = x.A + Tx * y.A;
  r.D = x.D + Tx * y.D;
  r.L = x.L + Tx * Tx * y.L + R(2) * Tx * (y.D * x.A - y.A * x.D);
  return r;
}

__device__ __forceinline__ void clamp_range(const int64_t* __restrict__ ro, int64_t r, int64_t n_seg,
                                            int64_t& k0, int64_t& k1) {
  k0 = ro[r];
  k1 = ro[r + 1];
  k0 = k0 < 0 ? 0 : (k0 > n_seg ? n_seg : k0);
  k1 = k1 < k0 ? k0 : (k1 > n_seg ? n_seg : k1);
}

// Rays with up to kCached segments are handled with all their tuples in registers.
constexpr int kCached = 8;

template <typename R>
__global__ __launch_bounds__(256) void merge_fwd_kernel(const float* __restrict__ seg_out,
                                                        int64_t n_seg,
                                                        const int64_t* __restrict__ ro,
                                                        const int64_t* __restrict__ ids,
                                                        int64_t n_rays, float* __restrict__ out) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  int64_t k0, k1;
  clamp_range(ro, r, n_seg, k0, k1);
  // Alg. 1/2 state: T(t_1 -> t_k) and C, A, D, L accumulated so far.
  R tau = 0, tlo = 0, Tpre = 1, cr = 0, cg = 0, cb = 0, A = 0, D = 0, L = 0;
  auto step = [&](const Tup<R>& x) {
    const R S = x.D * A - x.A * D;                    // Eq. 8
    L += Tpre * Tpre * x.L + R(2) * Tpre * S;         // Eq. 7
    cr += Tpre * x.cr; cg += Tpre * x.cg; cb += Tpre * x.cb;  // Eq. 3
    A += Tpre * x.A;                                  // Eq. 5
    D += Tpre * x.D;                                  // Eq. 6
    add_tau_t<R>(tau, tlo, x.tau, R(0));
    Tpre = exp_neg_t<R>(tau + tlo);                   // Eq. 4
  };
  const int64_t n = k1 - k0;
  if (n <= kCached) {
    // All of the ray's tuples are requested at once (two dependent loads in
    // flight per ray instead of two per segment).
    int64_t sid[kCached];
    Tup<R> x[kCached];
#pragma unroll
    for (int q = 0; q < kCached; ++q) {
      const int64_t s = q < n ? ids[k0 + q] : -1;
      sid[q] = (s >= 0 && s < n_seg) ? s : -1;
    }
#pragma unroll
    for (int q = 0; q < kCached; ++q)
      if (sid[q] >= 0) x[q] = load_tup<R>(seg_out, n_seg, sid[q]);
#pragma unroll
    for (int q = 0; q < kCached; ++q)
      if (sid[q] >= 0) step(x[q]);
  } else {
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t s = ids[k];
      if (s < 0 || s >= n_seg) continue;
      step(load_tup<R>(seg_out, n_seg, s));
    }
  }
  out[r] = static_cast<float>(Tpre);
  out[n_rays + r] = static_cast<float>(cr);
  out[2 * n_rays + r] = static_cast<float>(cg);
  out[3 * n_rays + r] = static_cast<float>(cb);
  out[4 * n_rays + r] = static_cast<float>(A);
  out[5 * n_rays + r] = static_cast<float>(D);
  out[6 * n_rays + r] = static_cast<float>(L);
}

// Gradient of P (+) x (+) S with respect to x, written to gseg[:, s].
template <typename R>
__device__ __forceinline__ void write_seg_grad(float* __restrict__ gseg, int64_t n_seg, int64_t s,
                                               const Tup<R>& P, R PT, const Tup<R>& x,
                                               const Tup<R>& Sk, R gT, R gCr, R gCg, R gCb, R gA,
                                               R gD, R gL) {
  const R Tk = exp_neg_t<R>(x.tau);
  const R ST = exp_neg_t<R>(Sk.tau + Sk.tlo);
  const R gA_k = PT * (gA + R(2) * gL * (PT * Tk * Sk.D - P.D));
  const R gD_k = PT * (gD + R(2) * gL * (P.A - PT * Tk * Sk.A));
  const R gL_k = gL * PT * PT;
  const R gT_k = PT * gT * ST + PT * (gCr * Sk.cr + gCg * Sk.cg + gCb * Sk.cb) +
                 (PT * gA - R(2) * gL * PT * P.D) * Sk.A +
                 (PT * gD + R(2) * gL * PT * P.A) * Sk.D +
                 gL * PT * PT * (R(2) * Tk * Sk.L + R(2) * (Sk.D * x.A - Sk.A * x.D));
  gseg[s] = static_cast<float>(-Tk * gT_k);
  gseg[n_seg + s] = static_cast<float>(PT * gCr);
  gseg[2 * n_seg + s] = static_cast<float>(PT * gCg);
  gseg[3 * n_seg + s] = static_cast<float>(PT * gCb);
  gseg[4 * n_seg + s] = static_cast<float>(gA_k);
  gseg[5 * n_seg + s] = static_cast<float>(gD_k);
  gseg[6 * n_seg + s] = static_cast<float>(gL_k);
}

template <typename R>
__global__ __launch_bounds__(256) void merge_bwd_kernel(const float* __restrict__ seg_out,
                                                        int64_t n_seg,
                                                        const int64_t* __restrict__ ro,
                                                        const int64_t* __restrict__ ids,
                                                        int64_t n_rays,
                                                        const float* __restrict__ gray,
                                                        float* __restrict__ gseg) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  int64_t k0, k1;
  clamp_range(ro, r, n_seg, k0, k1);
  const R gT = gray[r], gCr = gray[n_rays + r], gCg = gray[2 * n_rays + r],
          gCb = gray[3 * n_rays + r], gA = gray[4 * n_rays + r], gD = gray[5 * n_rays + r],
          gL = gray[6 * n_rays + r];
  if (k1 - k0 <= kCached) {
    Tup<R> x[kCached];
    int64_t sid[kCached];
#pragma unroll
    for (int q = 0; q < kCached; ++q) {
      const int64_t k = k0 + q;
      sid[q] = (k < k1) ? ids[k] : -1;
      const bool ok = sid[q] >= 0 && sid[q] < n_seg;
      if (!ok) sid[q] = -1;
      x[q] = ok ? load_tup<R>(seg_out, n_seg, sid[q]) : Tup<R>{0, 0, 0, 0, 0, 0, 0};
    }
    // Slots past the ray's last segment are skipped (by the whole wave when
    // no ray of it has that many); invalid ids inside it are identities.
    const int64_t n = k1 - k0;
    Tup<R> S[kCached];
    Tup<R> acc{0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = kCached - 1; q >= 0; --q) {
      if (q < n) {
        S[q] = acc;
        acc = fold<R>(x[q], exp_neg_t<R>(x[q].tau), acc);
      }
    }
    Tup<R> P{0, 0, 0, 0, 0, 0, 0};
    R PT = 1;
#pragma unroll
    for (int q = 0; q < kCached; ++q) {
      if (q < n) {
        if (sid[q] >= 0) write_seg_grad<R>(gseg, n_seg, sid[q], P, PT, x[q], S[q], gT, gCr, gCg, gCb, gA, gD, gL);
        P = fold<R>(P, PT, x[q]);
        PT = exp_neg_t<R>(P.tau + P.tlo);
      }
    }
    return;
  }
  // Reverse sweep: exclusive suffix fold of every segment, parked in gseg.
  Tup<R> S{0, 0, 0, 0, 0, 0, 0};
  for (int64_t k = k1 - 1; k >= k0; --k) {
    const int64_t s = ids[k];
    if (s < 0 || s >= n_seg) continue;
    gseg[s] = static_cast<float>(S.tau + S.tlo);
    gseg[n_seg + s] = static_cast<float>(S.cr);
    gseg[2 * n_seg + s] = static_cast<float>(S.cg);
    gseg[3 * n_seg + s] = static_cast<float>(S.cb);
    gseg[4 * n_seg + s] = static_cast<float>(S.A);
    gseg[5 * n_seg + s] = static_cast<float>(S.D);
    gseg[6 * n_seg + s] = static_cast<float>(S.L);
    const Tup<R> x = load_tup<R>(seg_out, n_seg, s);
    S = fold<R>(x, exp_neg_t<R>(x.tau), S);
  }
  // Forward sweep with the exclusive prefix fold P.
  Tup<R> P{0, 0, 0, 0, 0, 0, 0};
  R PT = 1;
  for (int64_t k = k0; k < k1; ++k) {
    const int64_t s = ids[k];
    if (s < 0 || s >= n_seg) continue;
    const Tup<R> x = load_tup<R>(seg_out, n_seg, s);
    const Tup<R> Sk = load_tup<R>(gseg, n_seg, s);
    write_seg_grad<R>(gseg, n_seg, s, P, PT, x, Sk, gT, gCr, gCg, gCb, gA, gD, gL);
    P = fold<R>(P, PT, x);
    PT = exp_neg_t<R>(P.tau + P.tlo);
  }
}

static inline unsigned grid_for(int64_t count, int block) {
  return static_cast<unsigned>((count + block - 1) / block);
}

hipError_t launch_merge_fwd(const float* seg_out, int64_t n_seg, const int64_t* ro,
                            const int64_t* ids, int64_t n_rays, float* out, bool fp64,
                            hipStream_t stream) {
  if (n_rays == 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(merge_fwd_kernel<double>, dim3(grid_for(n_rays, 256)), dim3(256), 0, stream,
                       seg_out, n_seg, ro, ids, n_rays, out);
  else
    hipLaunchKernelGGL(merge_fwd_kernel<float>, dim3(grid_for(n_rays, 256)), dim3(256), 0, stream,
                       seg_out, n_seg, ro, ids, n_rays, out);
  return hipGetLastError();
}

hipError_t launch_merge_bwd(const float* seg_out, int64_t n_seg, const int64_t* ro,
                            const int64_t* ids, int64_t n_rays, const float* gray, float* gseg,
                            bool fp64, hipStream_t stream) {
  if (n_rays == 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(merge_bwd_kernel<double>, dim3(grid_for(n_rays, 256)), dim3(256), 0, stream,
                       seg_out, n_seg, ro, ids, n_rays, gray, gseg);
  else
    hipLaunchKernelGGL(merge_bwd_kernel<float>, dim3(grid_for(n_rays, 256)), dim3(256), 0, stream,
                       seg_out, n_seg, ro, ids, n_rays, gray, gseg);
  return hipGetLastError();
}

// ---------------------------------------------------------------- input checks
// Codes: 1 seg_offsets[0] != 0, 2 seg_offsets[n_seg] != n, 3 seg_offsets
// decreasing, 4 t_end < t_start, 5 unsorted/overlapping intervals in a
// segment, 6 ray_offsets[0] != 0 or ray_offsets[n_rays] != n_seg,
// 7 ray_offsets decreasing, 8 seg_id out of range.  The smallest code wins.
__global__ void check_seg_kernel(const float* __restrict__ t0, const float* __restrict__ t1,
                                 int64_t n, const int64_t* __restrict__ off, int64_t n_seg,
                                 int* __restrict__ code) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s > n_seg) return;
  if (s == 0 && off[0] != 0) atomicMin(code, 1);
  if (s == n_seg) {
    if (off[n_seg] != n) atomicMin(code, 2);
    return;
  }
  const int64_t a = off[s], b = off[s + 1];
  if (b < a) {
    atomicMin(code, 3);
    return;
  }
  if (a < 0 || b > n) return;  // reported through codes 1-3
  for (int64_t i = a; i < b; ++i) {
    if (!(t1[i] >= t0[i])) atomicMin(code, 4);
    if (i > a && t0[i] < t1[i - 1]) atomicMin(code, 5);
  }
}

__global__ void check_ray_kernel(const int64_t* __restrict__ ro, const int64_t* __restrict__ ids,
                                 int64_t n_rays, int64_t n_seg, int* __restrict__ code) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r > n_rays) return;
  if ((r == 0 && ro[0] != 0) || (r == n_rays && ro[n_rays] != n_seg)) atomicMin(code, 6);
  if (r == n_rays) return;
  const int64_t a = ro[r], b = ro[r + 1];
  if (b < a) {
    atomicMin(code, 7);
    return;
  }
  if (a < 0 || b > n_seg) return;
  for (int64_t k = a; k < b; ++k)
    if (ids[k] < 0 || ids[k] >= n_seg) atomicMin(code, 8);
}

hipError_t launch_check(const SamplesDev& s, const int64_t* off, int64_t n_seg, const int64_t* ro,
                        const int64_t* ids, int64_t n_rays, int* code, hipStream_t stream) {
  hipLaunchKernelGGL(check_seg_kernel, dim3(grid_for(n_seg + 1, 256)), dim3(256), 0, stream, s.t0,
                     s.t1, s.n, off, n_seg, code);
  if (ro != nullptr && ids != nullptr)
    hipLaunchKernelGGL(check_ray_kernel, dim3(grid_for(n_rays + 1, 256)), dim3(256), 0, stream, ro,
                       ids, n_rays, n_seg, code);
  return hipGetLastError();
}

}  // namespace xl
