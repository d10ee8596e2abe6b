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
//
// When the caller gives the region boundaries of the tuple array, each
// workgroup first moves its rays' tuples into LDS with contiguous loads and
// folds from there (the region-aware form below); the gathering form above is
// the fallback for any layout.
#include "internal.h"
#include "xl_device.hpp"

// Multiply-adds are fused per source expression only (not across
// statements), so that the folds, inlined into the gathering and the
// region-aware kernels, round identically in both.
#pragma clang fp contract(on)

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

__device__ __forceinline__ Tup load_tup(const float* __restrict__ p, int64_t s) {
  const Tup7 t = load_tup7(p, s);
  return Tup{t.v[0], t.v[1], t.v[2], t.v[3], t.v[4], t.v[5], t.v[6]};
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

// Front-to-back fold of a ray's segment tuples (Alg. 1/2 state: T(t_1 -> t_k)
// and C, A, D, L accumulated so far).
template <typename R>
struct Fold {
  Depth<R> tau;
  float Tpre = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, A = 0.f, D = 0.f, L = 0.f;
  __device__ __forceinline__ void step(const Tup& x) {
    const float S = x.D * A - x.A * D;                 // Eq. 8
    L += Tpre * Tpre * x.L + 2.f * Tpre * S;           // Eq. 7
    cr += Tpre * x.cr; cg += Tpre * x.cg; cb += Tpre * x.cb;  // Eq. 3
    A += Tpre * x.A;                                   // Eq. 5
    D += Tpre * x.D;                                   // Eq. 6
    tau.add(x.tau);
    Tpre = tau.trans();                                // Eq. 4
  }
  __device__ __forceinline__ void store(float* __restrict__ out, int64_t n_rays, int64_t r) const {
    out[r] = Tpre;
    out[n_rays + r] = cr;
    out[2 * n_rays + r] = cg;
    out[3 * n_rays + r] = cb;
    out[4 * n_rays + r] = A;
    out[5 * n_rays + r] = D;
    out[6 * n_rays + r] = L;
  }
};

// Forward merge of ray r, tuples gathered from seg_out.
template <typename R>
__device__ __forceinline__ void fwd_gather_ray(const float* __restrict__ seg_out, int64_t n_seg,
                                               const int64_t* __restrict__ ro,
                                               const int64_t* __restrict__ ids, int64_t n_rays,
                                               float* __restrict__ out, int64_t r) {
  int64_t k0, k1;
  clamp_range(ro, r, n_seg, k0, k1);
  Fold<R> f;
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
      if (sid[q] >= 0) x[q] = load_tup(seg_out, sid[q]);
#pragma unroll
    for (int q = 0; q < kCached; ++q)
      if (sid[q] >= 0) f.step(x[q]);
  } else {
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t s = ids[k];
      if (s < 0 || s >= n_seg) continue;
      f.step(load_tup(seg_out, s));
    }
  }
  f.store(out, n_rays, r);
}

template <typename R>
__global__ __launch_bounds__(kMergeBlock) void merge_fwd_kernel(const float* __restrict__ seg_out,
                                                                int64_t n_seg,
                                                                const int64_t* __restrict__ ro,
                                                                const int64_t* __restrict__ ids,
                                                                int64_t n_rays,
                                                                float* __restrict__ out) {
  const int64_t r = merge_ray(n_rays);
  if (r >= n_rays) return;
  fwd_gather_ray<R>(seg_out, n_seg, ro, ids, n_rays, out, r);
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
__device__ __forceinline__ Tup seg_grad(float PT, float PA, float PD, const Tup& x,
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
  return Tup{-Tk * gT_k, PT * g.cr, PT * g.cg, PT * g.cb, gA_k, gD_k, gL_k};
}

template <typename R>
__device__ __forceinline__ void write_seg_grad(float* __restrict__ gseg, int64_t n_seg, int64_t s,
                                               float PT, float PA, float PD, const Tup& x,
                                               const Suffix<R>& S, const RayGrad& g) {
  const Tup d = seg_grad<R>(PT, PA, PD, x, S, g);
  store_tup7(gseg, s, d.tau, d.cr, d.cg, d.cb, d.A, d.D, d.L);
}

// Backward merge of ray r, tuples gathered from seg_out.  CACHED: rays of up
// to kCached segments keep their tuples and prefixes in registers (the
// same values as the parked form below, which the staged kernel's fallback
// uses alone to stay within its register budget).
template <typename R, bool CACHED = true>
__device__ __forceinline__ void bwd_gather_ray(const float* __restrict__ seg_out, int64_t n_seg,
                                               const int64_t* __restrict__ ro,
                                               const int64_t* __restrict__ ids, int64_t n_rays,
                                               const float* __restrict__ gray,
                                               float* __restrict__ gseg, int64_t r) {
  int64_t k0, k1;
  clamp_range(ro, r, n_seg, k0, k1);
  const RayGrad g{gray[r], gray[n_rays + r], gray[2 * n_rays + r], gray[3 * n_rays + r],
                  gray[4 * n_rays + r], gray[5 * n_rays + r], gray[6 * n_rays + r]};
  const int64_t n = k1 - k0;
  if (CACHED && n <= kCached) {
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
      x[q] = sid[q] >= 0 ? load_tup(seg_out, sid[q]) : Tup{0, 0, 0, 0, 0, 0, 0};
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
  // parked in the first three words of the segment's own gradient record.
  {
    Depth<R> ptau;
    float T = 1.f, A = 0.f, D = 0.f;
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t s = ids[k];
      if (s < 0 || s >= n_seg) continue;
      const Tup x = load_tup(seg_out, s);
      gseg[kTupStride * s] = T;
      gseg[kTupStride * s + 1] = A;
      gseg[kTupStride * s + 2] = D;
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
    const Tup x = load_tup(seg_out, s);
    const float PT = gseg[kTupStride * s], PA = gseg[kTupStride * s + 1], PD = gseg[kTupStride * s + 2];
    write_seg_grad<R>(gseg, n_seg, s, PT, PA, PD, x, S, g);
    S.push_front(x, exp_neg(x.tau));
  }
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
  bwd_gather_ray<R>(seg_out, n_seg, ro, ids, n_rays, gray, gseg, r);
}

// ---------------------------------------------------------------- region-aware form
// Region k's tuples are seg_out[:, roff[k] .. roff[k+1]) and, inside a region,
// the segments of consecutive rays are consecutive (the sample layout packs
// each region's segments in ray order).  The ids that a workgroup's
// kMergeBlock consecutive rays list therefore form one contiguous run per
// region.  The workgroup finds the runs (each id's region by binary search
// over the boundaries, then the lowest and highest id and the count per
// region), gives every listed tuple a slot in LDS, run after run, and moves
// the runs with contiguous loads (and, in the backward, the gradients back
// with contiguous stores).  Each lane then folds its ray from LDS.  A block
// whose ids break the assumption (a region's ids not contiguous, ids outside
// the boundaries, more listed ids than slots, decreasing ray offsets) merges
// its rays with the gathering form instead, so any layout gives the same
// result.
// LDS: the tuples of up to kCoopSlots listed ids (28 B each) plus 5 B of
// bookkeeping per slot and the region table, 39.6 KB with up to 64 regions:
// four workgroups per CU.  (256 consecutive rays of the K=64 workload list
// 1,079 ids on average, at most 1,168 in a sample of 256 blocks; a block
// over the slots gathers.)
constexpr int kMaxRegions = 256;
constexpr int kCoopSlots = 1152;

template <int RMAX>
struct CoopStage {
  int64_t roff[RMAX + 1];
  int lo[RMAX], hi[RMAX], cnt[RMAX];
  int base[RMAX + 1];
  int wsum[kMergeBlock / kWave];
  float tup[7][kCoopSlots];
  uint16_t slot[kCoopSlots];  // the listed id's slot
  int16_t kid[kCoopSlots];    // region of the listed id (-1: invalid id, skipped)
  uint8_t wrote[kCoopSlots];  // backward: the slot holds a gradient
  int fail;
};

// Largest k in [0, n) with a[k] <= v, for a[0] <= v (a non-decreasing).
template <typename T>
__device__ __forceinline__ int last_not_above(const T* a, int n, T v) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Fills st.tup with the tuples of the ids that the workgroup's rays list (ids
// [q0, q1) of the id array) and st.slot with each listed id's slot.  Returns
// false (for the whole workgroup) if the block must take the gathering form.
// Every thread handles the positions tid + i * kMergeBlock (i < kPerThread)
// and issues all of its global loads before it uses any, so that a workgroup
// waits for one round trip per phase, not one per position.
constexpr int kPerThread = (kCoopSlots + kMergeBlock - 1) / kMergeBlock;
static_assert(kMaxRegions <= kMergeBlock, "one thread per region in the count scan");
static_assert(kCoopSlots <= 65535, "16-bit slots");

template <int RMAX>
__device__ __forceinline__ bool coop_stage(CoopStage<RMAX>& st, const float* __restrict__ seg_out,
                                           int64_t n_seg, const int64_t* __restrict__ roff,
                                           int n_regions, const int64_t* __restrict__ ids,
                                           int64_t q0, int64_t q1, int64_t k0, int64_t k1,
                                           bool own, int64_t max_segs) {
  const int tid = threadIdx.x;
  const int n = static_cast<int>(q1 < q0 ? 0 : (q1 - q0 < kCoopSlots ? q1 - q0 : kCoopSlots));
  int64_t idv[kPerThread];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int p = tid + i * kMergeBlock;
    idv[i] = p < n ? ids[q0 + p] : -1;
  }
  if (tid <= n_regions) st.roff[tid] = roff[tid];
  if (tid < n_regions) {
    st.lo[tid] = INT32_MAX;
    st.hi[tid] = -1;
    st.cnt[tid] = 0;
  }
  if (tid == 0) st.fail = (q1 < q0 || q1 - q0 > kCoopSlots) ? 1 : 0;
  __syncthreads();
  // Every ray's range must lie inside the block's (ray offsets increasing).
  if (own && (k0 < q0 || k1 > q1 || k1 - k0 > max_segs)) st.fail = 1;
  const int64_t first = st.roff[0], last = st.roff[n_regions];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int p = tid + i * kMergeBlock;
    if (p < n) {
      const int64_t id = idv[i];
      int k = -1;
      if (id >= 0 && id < n_seg) {
        if (id < first || id >= last) {
          st.fail = 1;
        } else {
          k = last_not_above(st.roff, n_regions, id);
          const int64_t rel = id - st.roff[k];
          if (rel < 0 || rel > INT32_MAX - kCoopSlots) {  // (boundaries not increasing)
            st.fail = 1;
            k = -1;
          } else {
            atomicMin(&st.lo[k], static_cast<int>(rel));
            atomicMax(&st.hi[k], static_cast<int>(rel));
            atomicAdd(&st.cnt[k], 1);
          }
        }
      }
      st.kid[p] = static_cast<int16_t>(k);
    }
  }
  __syncthreads();
  // Contiguity per region, and the scan of the counts (run bases).
  {
    const int lane = tid % kWave, wave = tid / kWave;
    int c = 0;
    if (tid < n_regions) {
      c = st.cnt[tid];
      if (c > 0 && st.hi[tid] - st.lo[tid] + 1 != c) st.fail = 1;
    }
    int incl = c;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int y = __shfl_up(incl, d);
      if (lane >= d) incl += y;
    }
    if (lane == kWave - 1) st.wsum[wave] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += st.wsum[w];
    if (tid < n_regions) st.base[tid + 1] = before + incl;
    if (tid == 0) st.base[0] = 0;
  }
  __syncthreads();
  if (st.fail) return false;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int p = tid + i * kMergeBlock;
    if (p < n) {
      const int k = st.kid[p];
      if (k >= 0)
        st.slot[p] = static_cast<uint16_t>(st.base[k] + static_cast<int>(idv[i] - st.roff[k]) - st.lo[k]);
    }
  }
  // Contiguous loads, run after run: every load of the thread first, then
  // the LDS stores.
  const int used = st.base[n_regions];
  int64_t src[kPerThread];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int q = tid + i * kMergeBlock;
    src[i] = -1;
    if (q < used) {
      const int k = last_not_above(st.base, n_regions, q);
      src[i] = st.roff[k] + st.lo[k] + (q - st.base[k]);
    }
  }
  Tup7 v[kPerThread];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) v[i] = src[i] >= 0 ? load_tup7(seg_out, src[i]) : Tup7{};
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int q = tid + i * kMergeBlock;
    if (q < used) {
#pragma unroll
      for (int f = 0; f < 7; ++f) st.tup[f][q] = v[i].v[f];
    }
  }
  __syncthreads();
  return true;
}

template <int RMAX>
__device__ __forceinline__ Tup lds_tup(const CoopStage<RMAX>& st, int q) {
  return Tup{st.tup[0][q], st.tup[1][q], st.tup[2][q], st.tup[3][q],
             st.tup[4][q], st.tup[5][q], st.tup[6][q]};
}

// Rays of this workgroup: [r0, r1), the XCD-grouped block of merge_ray.
__device__ __forceinline__ void coop_rays(int64_t n_rays, int64_t& r0, int64_t& r1) {
  const int64_t nblocks = (n_rays + kMergeBlock - 1) / kMergeBlock;
  const int64_t per = (nblocks + kXcds - 1) / kXcds;
  const int64_t b = blockIdx.x;
  r0 = ((b % kXcds) * per + b / kXcds) * kMergeBlock;
  r1 = r0 + kMergeBlock < n_rays ? r0 + kMergeBlock : n_rays;
}

template <typename R, int RMAX>
__global__ __launch_bounds__(kMergeBlock) void merge_fwd_regions_kernel(
    const float* __restrict__ seg_out, int64_t n_seg, const int64_t* __restrict__ roff,
    int n_regions, const int64_t* __restrict__ ro, const int64_t* __restrict__ ids,
    int64_t n_rays, float* __restrict__ out) {
  __shared__ CoopStage<RMAX> st;
  int64_t r0, r1;
  coop_rays(n_rays, r0, r1);
  if (r0 >= n_rays) return;  // the whole workgroup
  const int64_t r = r0 + threadIdx.x;
  const bool own = r < r1;
  int64_t q0, q1, k0 = 0, k1 = 0, t;
  clamp_range(ro, r0, n_seg, q0, t);
  clamp_range(ro, r1 - 1, n_seg, t, q1);
  if (own) clamp_range(ro, r, n_seg, k0, k1);
  if (!coop_stage(st, seg_out, n_seg, roff, n_regions, ids, q0, q1, k0, k1, own, INT64_MAX)) {
    if (own) fwd_gather_ray<R>(seg_out, n_seg, ro, ids, n_rays, out, r);
    return;
  }
  if (!own) return;
  Fold<R> f;
  for (int64_t q = k0; q < k1; ++q) {
    const int p = static_cast<int>(q - q0);
    if (st.kid[p] >= 0) f.step(lds_tup(st, st.slot[p]));
  }
  f.store(out, n_rays, r);
}

// Backward of one ray from the staged tuples: the ray's positions are taken
// kStagedGroup at a time, last group first; for each group the prefix fold up to
// it is recomputed from LDS and the group's prefixes kept in registers, then
// the group is swept in reverse with the suffix fold, every gradient
// replacing its tuple.  Earlier groups are read before any of their slots is
// overwritten.  The arithmetic is that of the gathering form, step for step.
constexpr int kStagedGroup = 4;  // (keeps the backward within 128 VGPRs: four waves per SIMD)

template <typename R, int RMAX>
__device__ __forceinline__ void bwd_staged_ray(CoopStage<RMAX>& st, int64_t q0, int64_t k0,
                                               int64_t k1, const RayGrad& g) {
  Suffix<R> S;
  const int64_t n = k1 - k0;
  if (n <= 0) return;
  for (int64_t c0 = k0 + (n - 1) / kStagedGroup * kStagedGroup; c0 >= k0; c0 -= kStagedGroup) {
    Depth<R> ptau;
    float T = 1.f, A = 0.f, D = 0.f;
    for (int64_t q = k0; q < c0; ++q) {
      const int p = static_cast<int>(q - q0);
      if (st.kid[p] < 0) continue;
      const int s = st.slot[p];
      A += T * st.tup[4][s];
      D += T * st.tup[5][s];
      ptau.add(st.tup[0][s]);
      T = ptau.trans();
    }
    float PT[kStagedGroup], PA[kStagedGroup], PD[kStagedGroup];
    int sl[kStagedGroup];
    Tup x[kStagedGroup];
#pragma unroll
    for (int i = 0; i < kStagedGroup; ++i) {
      const int64_t q = c0 + i;
      sl[i] = -1;
      if (q < k1) {
        const int p = static_cast<int>(q - q0);
        if (st.kid[p] >= 0) {
          sl[i] = st.slot[p];
          x[i] = lds_tup(st, sl[i]);
          PT[i] = T; PA[i] = A; PD[i] = D;
          A += T * x[i].A;
          D += T * x[i].D;
          ptau.add(x[i].tau);
          T = ptau.trans();
        }
      }
    }
#pragma unroll
    for (int i = kStagedGroup - 1; i >= 0; --i) {
      if (sl[i] >= 0) {
        const Tup d = seg_grad<R>(PT[i], PA[i], PD[i], x[i], S, g);
        const int s = sl[i];
        st.tup[0][s] = d.tau; st.tup[1][s] = d.cr; st.tup[2][s] = d.cg; st.tup[3][s] = d.cb;
        st.tup[4][s] = d.A; st.tup[5][s] = d.D; st.tup[6][s] = d.L;
        st.wrote[s] = 1;
        S.push_front(x[i], exp_neg(x[i].tau));
      }
    }
  }
}

// Longest ray the staged backward takes (its regrouped prefixes cost
// O(n^2 / kStagedGroup)); a block with a longer ray gathers.
constexpr int64_t kStagedMaxSegs = 64;

template <typename R, int RMAX>
__global__ __launch_bounds__(kMergeBlock) void merge_bwd_regions_kernel(
    const float* __restrict__ seg_out, int64_t n_seg, const int64_t* __restrict__ roff,
    int n_regions, const int64_t* __restrict__ ro, const int64_t* __restrict__ ids,
    int64_t n_rays, const float* __restrict__ gray, float* __restrict__ gseg) {
  __shared__ CoopStage<RMAX> st;
  int64_t r0, r1;
  coop_rays(n_rays, r0, r1);
  if (r0 >= n_rays) return;
  const int64_t r = r0 + threadIdx.x;
  const bool own = r < r1;
  int64_t q0, q1, k0 = 0, k1 = 0, t;
  clamp_range(ro, r0, n_seg, q0, t);
  clamp_range(ro, r1 - 1, n_seg, t, q1);
  if (own) clamp_range(ro, r, n_seg, k0, k1);
  // Slots that no ray of the block writes (only if an id is listed twice,
  // outside the contract) are not stored.
  for (int q = threadIdx.x; q < kCoopSlots; q += kMergeBlock) st.wrote[q] = 0;
  // The ray's gradient is requested before the staging (its loads wait there).
  RayGrad g{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (own)
    g = RayGrad{gray[r], gray[n_rays + r], gray[2 * n_rays + r], gray[3 * n_rays + r],
                gray[4 * n_rays + r], gray[5 * n_rays + r], gray[6 * n_rays + r]};
  if (!coop_stage(st, seg_out, n_seg, roff, n_regions, ids, q0, q1, k0, k1, own, kStagedMaxSegs)) {
    if (own) bwd_gather_ray<R, false>(seg_out, n_seg, ro, ids, n_rays, gray, gseg, r);
    return;
  }
  if (own) bwd_staged_ray<R, RMAX>(st, q0, k0, k1, g);
  __syncthreads();
  // Contiguous stores, run after run.
  const int used = st.base[n_regions];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int q = threadIdx.x + i * kMergeBlock;
    if (q < used && st.wrote[q]) {
      const int k = last_not_above(st.base, n_regions, q);
      const int64_t id = st.roff[k] + st.lo[k] + (q - st.base[k]);
      store_tup7(gseg, id, st.tup[0][q], st.tup[1][q], st.tup[2][q], st.tup[3][q], st.tup[4][q],
                 st.tup[5][q], st.tup[6][q]);
    }
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

// The staged form needs the boundaries; by default it is taken from
// kStagedMinSegs segments up, where the tuples no longer stay in the caches
// and the gathering form is bound by its scattered 4-byte accesses (measured
// at 17.7M segments: forward 506 -> 362 us, backward 1163 -> 672 us).  Below
// that the gathering form is faster (at 0.76M segments 12 against 19 us
// forward): a workgroup's staging phases cost more latency than the gather.
constexpr int64_t kStagedMinSegs = int64_t(1) << 22;

static inline bool use_regions(const int64_t* roff, int n_regions, int64_t n_seg, bool force) {
  if (roff == nullptr || n_regions < 1 || n_regions > kMaxRegions) return false;
  return force || n_seg >= kStagedMinSegs;
}

template <typename R>
static void launch_fwd_regions(dim3 grid, const float* seg_out, int64_t n_seg, const int64_t* roff,
                               int n_regions, const int64_t* ro, const int64_t* ids, int64_t n_rays,
                               float* out, hipStream_t stream) {
  if (n_regions <= 64)
    hipLaunchKernelGGL((merge_fwd_regions_kernel<R, 64>), grid, dim3(kMergeBlock), 0, stream, seg_out,
                       n_seg, roff, n_regions, ro, ids, n_rays, out);
  else
    hipLaunchKernelGGL((merge_fwd_regions_kernel<R, kMaxRegions>), grid, dim3(kMergeBlock), 0, stream,
                       seg_out, n_seg, roff, n_regions, ro, ids, n_rays, out);
}

template <typename R>
static void launch_bwd_regions(dim3 grid, const float* seg_out, int64_t n_seg, const int64_t* roff,
                               int n_regions, const int64_t* ro, const int64_t* ids, int64_t n_rays,
                               const float* gray, float* gseg, hipStream_t stream) {
  if (n_regions <= 64)
    hipLaunchKernelGGL((merge_bwd_regions_kernel<R, 64>), grid, dim3(kMergeBlock), 0, stream, seg_out,
                       n_seg, roff, n_regions, ro, ids, n_rays, gray, gseg);
  else
    hipLaunchKernelGGL((merge_bwd_regions_kernel<R, kMaxRegions>), grid, dim3(kMergeBlock), 0, stream,
                       seg_out, n_seg, roff, n_regions, ro, ids, n_rays, gray, gseg);
}

hipError_t launch_merge_fwd(const float* seg_out, int64_t n_seg, const int64_t* roff,
                            int n_regions, const int64_t* ro, const int64_t* ids, int64_t n_rays,
                            float* out, bool fp64, bool staged, hipStream_t stream) {
  if (n_rays == 0) return hipSuccess;
  const dim3 grid(merge_grid(n_rays)), block(kMergeBlock);
  if (use_regions(roff, n_regions, n_seg, staged)) {
    if (fp64)
      launch_fwd_regions<double>(grid, seg_out, n_seg, roff, n_regions, ro, ids, n_rays, out, stream);
    else
      launch_fwd_regions<float>(grid, seg_out, n_seg, roff, n_regions, ro, ids, n_rays, out, stream);
  } else if (fp64) {
    hipLaunchKernelGGL(merge_fwd_kernel<double>, grid, block, kMergeLds, stream, seg_out, n_seg,
                       ro, ids, n_rays, out);
  } else {
    hipLaunchKernelGGL(merge_fwd_kernel<float>, grid, block, kMergeLds, stream, seg_out, n_seg,
                       ro, ids, n_rays, out);
  }
  return hipGetLastError();
}

hipError_t launch_merge_bwd(const float* seg_out, int64_t n_seg, const int64_t* roff,
                            int n_regions, const int64_t* ro, const int64_t* ids, int64_t n_rays,
                            const float* gray, float* gseg, bool fp64, bool staged,
                            hipStream_t stream) {
  if (n_rays == 0) return hipSuccess;
  const dim3 grid(merge_grid(n_rays)), block(kMergeBlock);
  if (use_regions(roff, n_regions, n_seg, staged)) {
    if (fp64)
      launch_bwd_regions<double>(grid, seg_out, n_seg, roff, n_regions, ro, ids, n_rays, gray, gseg,
                                 stream);
    else
      launch_bwd_regions<float>(grid, seg_out, n_seg, roff, n_regions, ro, ids, n_rays, gray, gseg,
                                stream);
  } else if (fp64) {
    hipLaunchKernelGGL(merge_bwd_kernel<double>, grid, block, kMergeLds, stream, seg_out, n_seg,
                       ro, ids, n_rays, gray, gseg);
  } else {
    hipLaunchKernelGGL(merge_bwd_kernel<float>, grid, block, kMergeLds, stream, seg_out, n_seg,
                       ro, ids, n_rays, gray, gseg);
  }
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
