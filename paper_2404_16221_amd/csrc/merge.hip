// Merge of segment tuples in ray order (Sec. 4.3, Eq. 3-8; App. A.2, Alg. 1-2).
//
// One lane per ray folds the ray's segments front to back.  The transmittance
// in front of segment k is the exclusive product of the segment
// transmittances (Eq. 4), formed as exp(-sum_{j<k} tau_j); the distortion
// loss gains 2 T_{<k} S_k + T_{<k}^2 L_k with S_k = D_k A_{<k} - A_k D_{<k}
// (Eq. 7-8).  Colour, opacity, depth and distortion are folded in float32.
// The running optical depth is a compensated float32 pair, or a float64
// (XL_MERGE_FP64), so that only the cross-segment transmittance product is
// wider than float32.
//
// The backward gives each segment the gradient of the merged tuple with
// respect to its own tuple only (the per-region differentiation rule of Sec.
// 4.2 and App. A.2): for segment k with exclusive prefix fold P and suffix fold
// S, the merged tuple is P (+) x_k (+) S, and the chain rule through the two
// (+) operations needs only P's transmittance, opacity and depth and all of S.
// A forward sweep records (P_T, P_A, P_D) of every segment; a reverse sweep
// carries S and writes the gradients.  Rays with up to kCached segments keep
// their tuples and prefixes in registers; longer rays park the prefixes in
// their own grad_seg entries, which the reverse sweep then overwrites.
//
// Rays are taken 256 to a workgroup, and consecutive workgroups of rays run
// on the same XCD: adjacent rays' segments are adjacent inside every region,
// so a cache line of tuples serves several neighbouring workgroups, which
// then find it in their XCD's L2.  Every tuple field is a separate 4-byte
// access (the tuples are region-major, a ray's segments in many regions), so
// the rays in flight on an XCD decide how many partly used lines its L2 must
// hold.  Each workgroup therefore reserves kMergeLds bytes of LDS it does not
// use, which holds two workgroups (two waves per SIMD) on a CU.
#include "internal.h"
#include "xl_device.hpp"

namespace xl {

constexpr int kMergeBlock = 256;
constexpr int kXcds = 8;  // MI355X: 8 XCDs, workgroups dispatched to them round robin
constexpr size_t kMergeLds = 64 * 1024;  // occupancy limit (see above)

// Running optical depth of a fold: float32 with TwoSum compensation, or float64.
template <typename R>
struct Depth;

template <>
struct Depth<float> {
  float hi = 0.f, lo = 0.f;
  __device__ __forceinline__ void add(float x) {  // Knuth's TwoSum, error kept in lo
    const float s = hi + x;
    const float bb = s - hi;
    lo += (hi - (s - bb)) + (x - bb);
    hi = s;
  }
  __device__ __forceinline__ float trans() const { return exp_neg(hi + lo); }
};

template <>
struct Depth<double> {
  double v = 0.0;
  __device__ __forceinline__ void add(float x) { v += static_cast<double>(x); }
  __device__ __forceinline__ float trans() const { return static_cast<float>(exp(-v)); }
};

struct Tup {
  float tau, cr, cg, cb, A, D, L;
};

__device__ __forceinline__ Tup load_tup(const float* __restrict__ p, int64_t n_seg, int64_t s) {
  Tup x;
  x.tau = p[s]; x.cr = p[n_seg + s]; x.cg = p[2 * n_seg + s]; x.cb = p[3 * n_seg + s];
  x.A = p[4 * n_seg + s]; x.D = p[5 * n_seg + s]; x.L = p[6 * n_seg + s];
  return x;
}

__device__ __forceinline__ void clamp_range(const int64_t* __restrict__ ro, int64_t r, int64_t n_seg,
                                            int64_t& k0, int64_t& k1) {
  k0 = ro[r];
  k1 = ro[r + 1];
  k0 = k0 < 0 ? 0 : (k0 > n_seg ? n_seg : k0);
  k1 = k1 < k0 ? k0 : (k1 > n_seg ? n_seg : k1);
}

// Ray of this thread: workgroup b of the launch takes ray block
// (b % kXcds) * per + b / kXcds, so each XCD walks a contiguous run of blocks.
__device__ __forceinline__ int64_t merge_ray(int64_t n_rays) {
  const int64_t nblocks = (n_rays + kMergeBlock - 1) / kMergeBlock;
  const int64_t per = (nblocks + kXcds - 1) / kXcds;
  const int64_t b = blockIdx.x;
  const int64_t lb = (b % kXcds) * per + b / kXcds;
  return lb * kMergeBlock + threadIdx.x;
}

// Rays with up to kCached segments are handled with all their tuples in registers.
constexpr int kCached = 8;

template <typename R>
__global__ __launch_bounds__(kMergeBlock) void merge_fwd_kernel(const float* __restrict__ seg_out,
                                                                int64_t n_seg,
                                                                const int64_t* __restrict__ ro,
                                                                const int64_t* __restrict__ ids,
                                                                int64_t n_rays,
                                                                float* __restrict__ out) {
  const int64_t r = merge_ray(n_rays);
  if (r >= n_rays) return;
  int64_t k0, k1;
  clamp_range(ro, r, n_seg, k0, k1);
  // Alg. 1/2 state: T(t_1 -> t_k) and C, A, D, L accumulated so far.
  Depth<R> tau;
  float Tpre = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, A = 0.f, D = 0.f, L = 0.f;
  auto step = [&](const Tup& x) {
    const float S = x.D * A - x.A * D;                 // Eq. 8
    L += Tpre * Tpre * x.L + 2.f * Tpre * S;           // Eq. 7
    cr += Tpre * x.cr; cg += Tpre * x.cg; cb += Tpre * x.cb;  // Eq. 3
    A += Tpre * x.A;                                   // Eq. 5
    D += Tpre * x.D;                                   // Eq. 6
    tau.add(x.tau);
    Tpre = tau.trans();                                // Eq. 4
  };
  const int64_t n = k1 - k0;
  if (n <= kCached) {
    // All of the ray's tuples are requested at once (two dependent loads in
    // flight per ray instead of two per segment).
    int64_t sid[kCached];
    Tup x[kCached];
#pragma unroll
    for (int q = 0; q < kCached; ++q) {
      const int64_t s = q < n ? ids[k0 + q] : -1;
      sid[q] = (s >= 0 && s < n_seg) ? s : -1;
    }
#pragma unroll
    for (int q = 0; q < kCached; ++q)
      if (sid[q] >= 0) x[q] = load_tup(seg_out, n_seg, sid[q]);
#pragma unroll
    for (int q = 0; q < kCached; ++q)
      if (sid[q] >= 0) step(x[q]);
  } else {
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t s = ids[k];
      if (s < 0 || s >= n_seg) continue;
      step(load_tup(seg_out, n_seg, s));
    }
  }
  out[r] = Tpre;
  out[n_rays + r] = cr;
  out[2 * n_rays + r] = cg;
  out[3 * n_rays + r] = cb;
  out[4 * n_rays + r] = A;
  out[5 * n_rays + r] = D;
  out[6 * n_rays + r] = L;
}

// Exclusive suffix fold of a ray's segments (everything behind segment k).
template <typename R>
struct Suffix {
  Depth<R> tau;
  float cr = 0.f, cg = 0.f, cb = 0.f, A = 0.f, D = 0.f, L = 0.f;
  // S <- x (+) S, x in front of S.
  __device__ __forceinline__ void push_front(const Tup& x, float Tx) {
    L = x.L + Tx * Tx * L + 2.f * Tx * (D * x.A - A * x.D);
    cr = x.cr + Tx * cr; cg = x.cg + Tx * cg; cb = x.cb + Tx * cb;
    A = x.A + Tx * A;
    D = x.D + Tx * D;
    tau.add(x.tau);
  }
};

struct RayGrad {
  float T, cr, cg, cb, A, D, L;
};

// Gradient of P (+) x (+) S with respect to x, written to gseg[:, s]; P enters
// through its transmittance PT, opacity PA and depth PD only.
template <typename R>
__device__ __forceinline__ void write_seg_grad(float* __restrict__ gseg, int64_t n_seg, int64_t s,
                                               float PT, float PA, float PD, const Tup& x,
                                               const Suffix<R>& S, const RayGrad& g) {
  const float Tk = exp_neg(x.tau);
  const float ST = S.tau.trans();
  const float gA_k = PT * (g.A + 2.f * g.L * (PT * Tk * S.D - PD));
  const float gD_k = PT * (g.D + 2.f * g.L * (PA - PT * Tk * S.A));
  const float gL_k = g.L * PT * PT;
  const float gT_k = PT * g.T * ST + PT * (g.cr * S.cr + g.cg * S.cg + g.cb * S.cb) +
                     (PT * g.A - 2.f * g.L * PT * PD) * S.A +
                     (PT * g.D + 2.f * g.L * PT * PA) * S.D +
                     g.L * PT * PT * (2.f * Tk * S.L + 2.f * (S.D * x.A - S.A * x.D));
  gseg[s] = -Tk * gT_k;
  gseg[n_seg + s] = PT * g.cr;
  gseg[2 * n_seg + s] = PT * g.cg;
  gseg[3 * n_seg + s] = PT * g.cb;
  gseg[4 * n_seg + s] = gA_k;
  gseg[5 * n_seg + s] = gD_k;
  gseg[6 * n_seg + s] = gL_k;
}

template <typename R>
__global__ __launch_bounds__(kMergeBlock) void merge_bwd_kernel(const float* __restrict__ seg_out,
                                                                int64_t n_seg,
                                                                const int64_t* __restrict__ ro,
                                                                const int64_t* __restrict__ ids,
                                                                int64_t n_rays,
                                                                const float* __restrict__ gray,
                                                                float* __restrict__ gseg) {
  const int64_t r = merge_ray(n_rays);
  if (r >= n_rays) return;
  int64_t k0, k1;
  clamp_range(ro, r, n_seg, k0, k1);
  const RayGrad g{gray[r], gray[n_rays + r], gray[2 * n_rays + r], gray[3 * n_rays + r],
                  gray[4 * n_rays + r], gray[5 * n_rays + r], gray[6 * n_rays + r]};
  const int64_t n = k1 - k0;
  if (n <= kCached) {
    Tup x[kCached];
    int64_t sid[kCached];
#pragma unroll
    for (int q = 0; q < kCached; ++q) {
      const int64_t s = q < n ? ids[k0 + q] : -1;
      sid[q] = (s >= 0 && s < n_seg) ? s : -1;
    }
    // Invalid ids inside the ray are identities (zero tuples).
#pragma unroll
    for (int q = 0; q < kCached; ++q)
      x[q] = sid[q] >= 0 ? load_tup(seg_out, n_seg, sid[q]) : Tup{0, 0, 0, 0, 0, 0, 0};
    // Forward sweep: exclusive prefix transmittance, opacity and depth.  Slots
    // past the ray's last segment are skipped (by the whole wave when no ray
    // of it has that many).
    float PT[kCached], PA[kCached], PD[kCached];
    Depth<R> ptau;
    float T = 1.f, A = 0.f, D = 0.f;
#pragma unroll
    for (int q = 0; q < kCached; ++q) {
      if (q < n) {
        PT[q] = T; PA[q] = A; PD[q] = D;
        A += T * x[q].A;
        D += T * x[q].D;
        ptau.add(x[q].tau);
        T = ptau.trans();
      }
    }
    // Reverse sweep with the exclusive suffix fold.
    Suffix<R> S;
#pragma unroll
    for (int q = kCached - 1; q >= 0; --q) {
      if (q < n) {
        if (sid[q] >= 0) write_seg_grad<R>(gseg, n_seg, sid[q], PT[q], PA[q], PD[q], x[q], S, g);
        S.push_front(x[q], exp_neg(x[q].tau));
      }
    }
    return;
  }
  // Forward sweep: the exclusive prefix (P_T, P_A, P_D) of every segment,
  // parked in the segment's own tau, A and D gradient entries.
  {
    Depth<R> ptau;
    float T = 1.f, A = 0.f, D = 0.f;
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t s = ids[k];
      if (s < 0 || s >= n_seg) continue;
      const Tup x = load_tup(seg_out, n_seg, s);
      gseg[s] = T;
      gseg[4 * n_seg + s] = A;
      gseg[5 * n_seg + s] = D;
      A += T * x.A;
      D += T * x.D;
      ptau.add(x.tau);
      T = ptau.trans();
    }
  }
  // Reverse sweep: the suffix fold S, and every segment's gradient.
  Suffix<R> S;
  for (int64_t k = k1 - 1; k >= k0; --k) {
    const int64_t s = ids[k];
    if (s < 0 || s >= n_seg) continue;
    const Tup x = load_tup(seg_out, n_seg, s);
    const float PT = gseg[s], PA = gseg[4 * n_seg + s], PD = gseg[5 * n_seg + s];
    write_seg_grad<R>(gseg, n_seg, s, PT, PA, PD, x, S, g);
    S.push_front(x, exp_neg(x.tau));
  }
}

static inline unsigned merge_grid(int64_t n_rays) {
  const int64_t nblocks = (n_rays + kMergeBlock - 1) / kMergeBlock;
  const int64_t per = (nblocks + kXcds - 1) / kXcds;
  return static_cast<unsigned>(per * kXcds);
}

static inline unsigned grid_for(int64_t count, int block) {
  return static_cast<unsigned>((count + block - 1) / block);
}

hipError_t launch_merge_fwd(const float* seg_out, int64_t n_seg, const int64_t* ro,
                            const int64_t* ids, int64_t n_rays, float* out, bool fp64,
                            hipStream_t stream) {
  if (n_rays == 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(merge_fwd_kernel<double>, dim3(merge_grid(n_rays)), dim3(kMergeBlock),
                       kMergeLds, stream, seg_out, n_seg, ro, ids, n_rays, out);
  else
    hipLaunchKernelGGL(merge_fwd_kernel<float>, dim3(merge_grid(n_rays)), dim3(kMergeBlock),
                       kMergeLds, stream, seg_out, n_seg, ro, ids, n_rays, out);
  return hipGetLastError();
}

hipError_t launch_merge_bwd(const float* seg_out, int64_t n_seg, const int64_t* ro,
                            const int64_t* ids, int64_t n_rays, const float* gray, float* gseg,
                            bool fp64, hipStream_t stream) {
  if (n_rays == 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(merge_bwd_kernel<double>, dim3(merge_grid(n_rays)), dim3(kMergeBlock),
                       kMergeLds, stream, seg_out, n_seg, ro, ids, n_rays, gray, gseg);
  else
    hipLaunchKernelGGL(merge_bwd_kernel<float>, dim3(merge_grid(n_rays)), dim3(kMergeBlock),
                       kMergeLds, stream, seg_out, n_seg, ro, ids, n_rays, gray, gseg);
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
