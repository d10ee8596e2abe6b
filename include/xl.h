/*
 * xl.h -- C ABI of the partitioned volume renderer (NeRF-XL, arXiv 2404.16221)
 * for AMD Instinct MI355X (gfx950).
 *
 * The method (Sec. 4.3): each of K disjoint axis-aligned regions composites
 * the samples it owns along every ray into a per-segment partial tuple; the
 * tuples of one ray are then merged front to back with an exclusive product of
 * the segment transmittances (Eq. 3-8).  The merge equals single-pass
 * rendering exactly (App. B.1).  Here the K regions are K shares of one GPU.
 *
 * Conventions for every entry point:
 *   - Pointers marked "device" are HIP device memory owned by the caller; the
 *     library never frees or retains them.  Sample arrays must be 16-byte
 *     aligned.  `stream` is a hipStream_t passed as void* (NULL = null stream).
 *   - Compute calls are asynchronous on `stream`, allocate nothing, and never
 *     synchronise the device.  Argument errors are detected on the host before
 *     anything is launched.
 *   - Return value: XL_OK (0) or a negative error code; xl_last_error() gives
 *     a message for the calling thread.
 *   - Sample layout (Sec. 4.2: each region holds the samples that fall in its
 *     axis-aligned box): samples of all regions packed
 *     region-major; segment s owns samples [seg_offsets[s], seg_offsets[s+1]),
 *     which belong to one ray and one region, sorted by t, with
 *     non-overlapping intervals [t_start, t_end].  Density sigma >= 0 with
 *     every optical depth sigma * (t_end - t_start) finite (the wave scans
 *     scale partial sums by 0 and 1 instead of selecting between them);
 *     colour and interval ends in any finite range.
 *   - Segment tuple (what each region reduces its samples to before any
 *     exchange, App. A.2):
 *     seg_out is float32 [n_seg][XL_TUPLE_STRIDE]: one 32-byte record per
 *     segment (array 16-byte aligned), words
 *       0 tau = sum sigma_i delta_i  (segment transmittance is exp(-tau))
 *       1-3 C = sum w_i c_i, 4 A = sum w_i, 5 D = sum w_i m_i (unnormalised),
 *       6 L = sum_ij w_i w_j |m_i - m_j| + 1/3 sum_i w_i^2 delta_i,
 *       7 zero (written as 0, ignored when read);
 *     gradients with respect to the tuples (grad_seg) use the same records.
 *     with delta_i = t_end - t_start, m_i the interval midpoint, alpha_i =
 *     1 - exp(-sigma_i delta_i), w_i = alpha_i prod_{j<i} (1 - alpha_j) taken
 *     inside the segment (transmittance starts at 1).  An empty segment has
 *     the identity tuple (all zeros).
 *   - Ray tuple: ray_out is float32 [7][n_rays] = (T, r, g, b, A, D, L) of the
 *     whole ray (Eq. 3-7); a ray with no segments gives (1, 0, ..., 0).
 */
#ifndef XL_H
#define XL_H

/* Words per segment tuple record (seg_out, grad_seg); see the conventions. */
#define XL_TUPLE_STRIDE 8

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define XL_OK 0
#define XL_PENDING 1
#define XL_EINVAL (-1)
#define XL_ENOMEM (-2)
#define XL_EHIP (-3)
#define XL_EAGAIN (-4)
#define XL_EFAULT (-5)

/* Storage type of sigma and rgb (and of their gradients).  t_start/t_end are
 * always float32; accumulation is always float32 or wider.  XL_BF16_F16 keeps
 * sigma (and dl/dsigma) in bfloat16 and rgb (and dl/drgb) in float16: the
 * same two bytes per value, with colour rounded to 2^-11 relative instead of
 * bfloat16's 2^-8 (accepted by the segment and generator entry points and the
 * server; the feature and breakable entry points take one storage type). */
#define XL_F32 0
#define XL_BF16 1
#define XL_F16 2
#define XL_BF16_F16 3

/* xl_merge_* flags. */
#define XL_MERGE_FP64 1   /* the running optical depth in float64 */
#define XL_MERGE_STAGED 2 /* with region_offsets: the LDS-staged form at any size */

typedef struct xl_samples {
  int32_t dtype;        /* XL_F32, XL_BF16, XL_F16 or XL_BF16_F16 */
  const void* sigma;    /* device [n] densities */
  const void* rgb;      /* device [n][3] colours */
  const float* t_start; /* device [n] interval starts */
  const float* t_end;   /* device [n] interval ends */
  int64_t n;            /* number of samples (>= 0) */
} xl_samples;

/* Library version (major * 10000 + minor * 100 + patch). */
int xl_version(void);

/* Message describing the last error on this thread ("" if none). */
const char* xl_last_error(void);

/* Bytes of device workspace that xl_render_segments_fwd fills and
 * xl_render_segments_bwd reads for n samples (per-tile partial tuples and
 * carries; about 0.41 byte per sample). */
size_t xl_segments_workspace_bytes(int64_t n);

/*
 * Per-segment composite, forward (Sec. 4.3: each region first reduces its own
 * samples to one partial tuple per ray segment; Eq. 1-2 evaluated per segment).
 *   s            samples (device arrays, see conventions)
 *   seg_offsets  device int64 [n_seg + 1], non-decreasing, seg_offsets[0] = 0,
 *                seg_offsets[n_seg] = s->n
 *   seg_out      device float32 [n_seg][XL_TUPLE_STRIDE], 16-byte aligned,
 *                written (every segment)
 *   workspace    device, >= xl_segments_workspace_bytes(s->n) bytes, written;
 *                keep it unchanged for the matching backward call
 * Errors: XL_EINVAL for null pointers, bad dtype, negative sizes, misaligned
 * sample arrays or seg_out, or a workspace that is too small; XL_EHIP if a
 * launch fails.
 */
int xl_render_segments_fwd(const xl_samples* s, const int64_t* seg_offsets, int64_t n_seg,
                           float* seg_out, void* workspace, size_t workspace_bytes,
                           void* stream);

/*
 * Per-segment composite, forward, allocating nothing and taking no workspace.
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, kernels and results as xl_render_segments_fwd, except that the
 * tile records go to a static device array of XL_STATIC_SCRATCH_BYTES per GPU,
 * held by the library until the process ends.  Hence:
 *   - at most 168,427,520 samples per call (xl_segments_workspace_bytes(n)
 *     <= XL_STATIC_SCRATCH_BYTES); larger calls fail with XL_EINVAL before
 *     anything is launched;
 *   - every call on one GPU shares that array: calls that overlap on one GPU
 *     (concurrent streams or threads) race and give wrong tuples; serialise
 *     them;
 *   - no xl_render_segments_bwd can follow (it needs the workspace of
 *     xl_render_segments_fwd), so this is a forward-only (inference) call.
 * The current device must be the device of `stream` and of the arrays.  The
 * first call on a device looks up the array's address (hipGetSymbolAddress);
 * XL_EHIP if that fails.  Nothing is zeroed: every record is written before it
 * is read within the call.
 */
#define XL_STATIC_SCRATCH_BYTES (64u << 20)
int xl_render_segments_fwd_static(const xl_samples* s, const int64_t* seg_offsets,
                                  int64_t n_seg, float* seg_out, void* stream);

/*
 * Per-segment composite, backward.  Given grad_seg = dl/d(seg tuple) (device
 * float32 [n_seg][XL_TUPLE_STRIDE], 16-byte aligned, word 0 is dl/dtau, word 7
 * ignored), writes dl/dsigma (device [n])
 * and dl/drgb (device [n][3]) in the storage dtype of `s`, overwriting them.
 * Transmittance is recomputed (forward and reverse wave scans); nothing per
 * sample is kept from the forward.  `workspace` must hold what the forward
 * call on the same inputs wrote.  Errors as for the forward.
 */
int xl_render_segments_bwd(const xl_samples* s, const int64_t* seg_offsets, int64_t n_seg,
                           const void* workspace, size_t workspace_bytes,
                           const float* grad_seg, void* grad_sigma, void* grad_rgb,
                           void* stream);

/*
 * Merge of segment tuples in ray order (Eq. 3-8; Alg. 1 and 2 of App. A.2
 * with Eq. 7's factor 2 and each segment's own A, D in the cross term).
 *   seg_out         device float32 [n_seg][XL_TUPLE_STRIDE] from
 *                   xl_render_segments_fwd (16-byte aligned)
 *   region_offsets  device int64 [n_regions + 1] or NULL: region k's tuples
 *                   are records region_offsets[k] .. region_offsets[k+1] - 1
 *                   (the sample layout packs each region's segments in ray
 *                   order, so consecutive rays list consecutive tuples of
 *                   each region).  Given (1 <= n_regions <= 256) and from
 *                   4,194,304 segments up (at any size with
 *                   XL_MERGE_STAGED), each workgroup of 256 rays moves its
 *                   rays' tuples into LDS run by run with contiguous loads
 *                   (and the gradients back with contiguous stores) before
 *                   folding.  Otherwise, and for a workgroup whose ids do not
 *                   form one contiguous run per region (or that lists more
 *                   than 1,280 ids, or, backward, has a ray of more than 64
 *                   segments), every ray gathers its own tuples: below that
 *                   size the tuples stay in the caches and gathering is
 *                   faster.  The result is the same either way.
 *   n_regions       entries of region_offsets minus one (ignored if NULL)
 *   ray_offsets     device int64 [n_rays + 1]; ray r's segments are
 *                   seg_ids[ray_offsets[r] .. ray_offsets[r+1]) front to back
 *                   (the paper's ordered index list I)
 *   seg_ids         device int64 [n_seg], values in [0, n_seg); ids outside
 *                   are skipped (identities); each segment is listed at most
 *                   once
 *   ray_out         device float32 [7][n_rays], written
 *   flags           XL_MERGE_FP64 (the running optical depth, i.e. the
 *                   cross-segment transmittance product, in float64; the
 *                   other fields fold in float32 either way) and/or
 *                   XL_MERGE_STAGED
 * Errors: XL_EINVAL for negative counts, unknown flags, NULL arrays, or
 * region_offsets given with n_regions < 1.
 */
int xl_merge_fwd(const float* seg_out, int64_t n_seg, const int64_t* region_offsets,
                 int32_t n_regions, const int64_t* ray_offsets, const int64_t* seg_ids,
                 int64_t n_rays, float* ray_out, int32_t flags, void* stream);

/*
 * Merge, backward: grad_ray = dl/d(T, r, g, b, A, D, L) (device float32
 * [7][n_rays]) -> grad_seg = dl/d(tau, r, g, b, A, D, L) of every segment
 * listed in seg_ids (device float32 [n_seg][XL_TUPLE_STRIDE], 16-byte aligned;
 * the records of listed segments are overwritten, word 7 with 0, and the
 * records of segments that no ray lists are left untouched).  Each segment is listed by
 * at most one ray.  Exclusive prefix and suffix folds per ray; the paper's
 * rule that each region differentiates only through its own tuple (Sec. 4.2,
 * App. A.2) is exactly this per-segment Jacobian.  Arguments as for the
 * forward.
 */
int xl_merge_bwd(const float* seg_out, int64_t n_seg, const int64_t* region_offsets,
                 int32_t n_regions, const int64_t* ray_offsets, const int64_t* seg_ids,
                 int64_t n_rays, const float* grad_ray, float* grad_seg, int32_t flags,
                 void* stream);

/*
 * Input validation (synchronous; for debugging and tests).  Checks on the
 * device that seg_offsets is non-decreasing from 0 to n, every interval has
 * t_end >= t_start, intervals inside a segment are sorted and disjoint,
 * ray_offsets is non-decreasing from 0 to n_seg and seg_ids are in range.
 * Returns XL_OK or XL_EINVAL with a message naming the first failed check.
 * ray_offsets/seg_ids may be NULL (then n_rays is ignored).
 */
int xl_check_inputs(const xl_samples* s, const int64_t* seg_offsets, int64_t n_seg,
                    const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                    void* stream);

/*
 * Synthetic workload generator on the device (the stand-in for per-region
 * NeRF evaluation): rays [ray0, ray0 + n_rays) of a seeded workload, packed
 * region-major exactly as the input contract above requires.  Bit-identical
 * to the host generator (synth.py) in every sample and in the layout.  grid[0]*grid[1]*grid[2] <= 256 regions,
 * grid[0]+grid[1]+grid[2] <= 18.
 */
typedef struct xl_gen_params {
  int64_t n_rays;    /* rays to generate */
  int64_t ray0;      /* index of the first ray in the workload */
  int32_t n_min;     /* samples per ray, uniform in [n_min, n_max] */
  int32_t n_max;
  int32_t grid[3];   /* regions: a gx x gy x gz grid over [-1, 1]^3 */
  int32_t reserved;
  double sigma_mu;   /* density lognormal(mu, s) */
  double sigma_s;
  double zero_frac;  /* fraction of densities set to 0 */
  double width_mean; /* mean interval width (exponential) */
  double t_far;      /* rays span [0, t_far] */
  uint64_t seed;
} xl_gen_params;

/* Device workspace bytes for xl_gen_plan / xl_gen_fill. */
size_t xl_gen_workspace_bytes(const xl_gen_params* p);

/* Phase 1 (synchronises `stream`): ray structure and layout into the
 * workspace; returns the number of samples and segments to allocate. */
int xl_gen_plan(const xl_gen_params* p, void* workspace, size_t workspace_bytes,
                int64_t* n_samples, int64_t* n_seg, void* stream);

/* Phase 2 (asynchronous): samples in storage type `dtype` and the CSR arrays
 * (seg_offsets [n_seg+1], ray_offsets [n_rays+1], seg_ids [n_seg]) and
 * region_offsets [K+1] (K = grid[0]*grid[1]*grid[2]: the first segment of
 * each region, then n_seg; the merge's region boundaries), any of the four
 * may be NULL, from the workspace filled by xl_gen_plan with the same
 * parameters. */
int xl_gen_fill(const xl_gen_params* p, int32_t dtype, void* workspace, size_t workspace_bytes,
                int64_t n_seg, void* sigma, void* rgb, float* t_start, float* t_end,
                int64_t* seg_offsets, int64_t* ray_offsets, int64_t* seg_ids,
                int64_t* region_offsets, void* stream);

/*
 * Spatial partitioning (Sec. 4.4, App. A.3), on the host.  Splits space
 * `levels` times (0 <= levels <= 6, so K = 2^levels <= 64 boxes) at planes
 * where the per-axis CDF of `points` reaches one half: at each node, for each
 * axis, the plane is the node's point coordinate of rank floor(m/2) (0-based,
 * m points; a node without points takes the middle of its box), and the axis
 * kept is the one whose two children have the smaller worst aspect ratio
 * (longest over shortest extent, extents clipped to the bounding box of all
 * points; ties go to x, then y).  Points below the plane go to the low child.
 *   points  host float32 [n_points][3], finite
 *   axis    host int32 [K - 1], written: split axis (0, 1, 2) of each node
 *   plane   host float32 [K - 1], written: split coordinate of each node
 * The tree is heap-ordered: node i has children 2i+1 (coordinate < plane)
 * and 2i+2 (coordinate >= plane); box b is leaf node b + K - 1.  The
 * outermost boxes extend to infinity.  Errors: XL_EINVAL for levels out of
 * range, n_points < 0, NULL arrays or a non-finite point.  Synchronous; no
 * device work.
 */
int xl_partition_build(const float* points, int64_t n_points, int32_t levels, int32_t* axis,
                       float* plane);

/* Rays and their samples before distribution, ray-major (device arrays). */
typedef struct xl_rays {
  const float* origins;        /* device float32 [n_rays][3] */
  const float* dirs;           /* device float32 [n_rays][3] (any length, not all 0) */
  const float* t_start;        /* device float32 [n] */
  const float* t_end;          /* device float32 [n] */
  const int64_t* ray_offsets;  /* device int64 [n_rays + 1]: ray r owns samples
                                  [ray_offsets[r], ray_offsets[r+1]), sorted:
                                  t_start <= t_end <= next t_start */
  int64_t n_rays;
} xl_rays;

/* Device workspace bytes for xl_pack_plan / xl_pack_fill: about
 * 18 * 2^levels + 16 bytes per ray (10 * 2^levels + 16 above 16 boxes).
 * One ray's run of samples in one box is limited to 134,217,727 samples
 * (2^31 / 16); a longer run keeps only its first that many. */
size_t xl_pack_workspace_bytes(int64_t n_rays, int32_t levels);

/*
 * Sample distribution (Sec. 4.2), phase 1 (synchronises `stream`).  Cuts every
 * sample interval at the points where its ray crosses a face of the boxes of
 * the tree (axis, plane: device copies of xl_partition_build's output),
 * tags the pieces with their box and plans their region-major layout.  Box
 * b's interval on a ray is [t_in, t_out) from a float64 slab test, each face
 * parameter being (face - origin) / direction, rounded to float32; the piece
 * of sample [s, e) is [max(s, t_in), min(e, t_out)) when that has positive
 * length; a zero-length sample stays whole in the box whose interval holds s.
 * Returns the number of pieces and of segments (one per ray and box with
 * pieces) to allocate.  Errors: XL_EINVAL for NULL arrays, levels out of range
 * or a small workspace; XL_EHIP for launch or copy failures.
 */
int xl_pack_plan(const xl_rays* rays, const int32_t* axis, const float* plane, int32_t levels,
                 void* workspace, size_t workspace_bytes, int64_t* n_pieces, int64_t* n_seg,
                 void* stream);

/*
 * Phase 2 (asynchronous), from the workspace that xl_pack_plan filled for the
 * same rays and tree: writes the pieces in the sample layout of the composite
 * calls above -- t_start, t_end [n_pieces], seg_offsets [n_seg + 1], box b's
 * segments (rays in order) before box b+1's -- plus ray_offsets [n_rays + 1]
 * and seg_ids [n_seg] listing each ray's segments front to back.  Optional
 * (may be NULL): src [n_pieces] int64, the input sample each piece comes from
 * (for evaluating the owning region's field there), seg_box [n_seg] int32,
 * and region_offsets [2^levels + 1] int64 (box b's segments are
 * [region_offsets[b], region_offsets[b+1]); the merge's region boundaries).
 * n_seg must be the plan's.  Samples that break the sortedness contract give
 * unspecified pieces, never stores outside these arrays.
 */
int xl_pack_fill(const xl_rays* rays, const int32_t* axis, const float* plane, int32_t levels,
                 void* workspace, size_t workspace_bytes, int64_t n_seg, float* t_start,
                 float* t_end, int64_t* src, int64_t* seg_offsets, int64_t* ray_offsets,
                 int64_t* seg_ids, int32_t* seg_box, int64_t* region_offsets, void* stream);

/*
 * Feature channels (App. B.2: breakable integrals are closed under integration
 * against a breakable factor, Property 2; with the transmittance as that
 * factor every per-sample feature vector f_i rendered with the volume-rendering
 * weights splits over regions like colour).  Per segment k, Phi_k =
 * sum_i w_i f_i with the weights of the colour path (transmittance from 1 at
 * the segment start); per ray, Phi = sum_k exp(-sum_{j<k} tau_j) Phi_k front
 * to back.  Uses: semantic logits, normals, learned features, or the squared
 * depth of a variance estimate.
 */
typedef struct xl_features {
  int32_t dtype;        /* storage of sigma, feat and their gradients */
  int32_t n_feat;       /* F: 4, 8, 16 or 32 channels */
  const void* sigma;    /* device [n] */
  const void* feat;     /* device [n][F], 16-byte aligned */
  const float* t_start; /* device [n] */
  const float* t_end;   /* device [n] */
  int64_t n;
} xl_features;

/* Per segment: phi_seg float32 [F][n_seg] (written), and tau_seg float32
 * [n_seg], the segment's optical depth (written; may be NULL).  Samples and
 * seg_offsets as for xl_render_segments_fwd.  FP32 accumulation. */
int xl_render_features_fwd(const xl_features* f, const int64_t* seg_offsets, int64_t n_seg,
                           float* phi_seg, float* tau_seg, void* stream);

/* Per ray: phi_ray float32 [F][n_rays] from tau_seg and phi_seg in the order
 * of ray_offsets / seg_ids (as for xl_merge_fwd; a ray without segments gets
 * zeros). */
int xl_merge_features_fwd(const float* tau_seg, const float* phi_seg, int32_t n_feat, int64_t n_seg,
                          const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                          float* phi_ray, void* stream);

/* Backward of the merge: grad_ray = dl/dphi_ray [F][n_rays] -> grad_phi_seg
 * [F][n_seg] = T_{<k} grad_ray and grad_tau_seg [n_seg] = -sum over later
 * segments of T_{<k'} (grad_ray . phi_k'), for every listed segment (each
 * listed by at most one ray; unlisted entries are left untouched). */
int xl_merge_features_bwd(const float* tau_seg, const float* phi_seg, int32_t n_feat, int64_t n_seg,
                          const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                          const float* grad_ray, float* grad_phi_seg, float* grad_tau_seg,
                          void* stream);

/* Backward per segment: dl/dsigma [n] and dl/dfeat [n][F] in the storage
 * dtype.  grad_tau_seg may be NULL (no gradient through later segments).
 * accumulate_sigma = 1 adds to grad_sigma (e.g. the colour path's), 0
 * overwrites it; grad_feat is always overwritten.  Transmittance is
 * recomputed; phi_seg is the forward's output for the same samples. */
int xl_render_features_bwd(const xl_features* f, const int64_t* seg_offsets, int64_t n_seg,
                           const float* phi_seg, const float* grad_phi_seg,
                           const float* grad_tau_seg, void* grad_sigma, void* grad_feat,
                           int32_t accumulate_sigma, void* stream);

/*
 * Breakable integrals composited across regions (App. B.2): the family that
 * Property 2 (integration against a breakable factor) and Property 1
 * (products) generate from the transmittance, up to one level of nesting.
 * With F per-sample channels f_c and P pairs (a_p, b_p) of them, and
 * w = T sigma the volume-rendering weight:
 *   first order   Phi_c = int w f_c  (colour, opacity, depth, features ...)
 *   second order  Psi_p = int w(u) f_a(u) [int_{v<u} w(v) f_b(v) dv] du
 *                 (the distortion loss of App. B.2's Examples is
 *                 2 (Psi_(m,1) - Psi_(1,m)) plus its within-sample term).
 * Quadrature as xl_render_segments_fwd's (piecewise-constant density and
 * channels per sample interval): Phi_c = sum_i w_i f_ci, Psi_p = sum_i w_i a_i
 * sum_{j<i} w_j b_j + 1/2 sum_i w_i^2 a_i b_i.
 * Tuples are float32 structure of arrays with 1 + F + P rows: per segment
 * (tau, Phi, Psi) with T from 1 inside the segment, per ray (T, Phi, Psi).
 * A ray's segments fold front to back by
 *   (x (+) y) = (tau_x + tau_y, Phi_x + T_x Phi_y,
 *                Psi_x + T_x^2 Psi_y + T_x Phi_(a)y Phi_(b)x).
 * Channel sources: XL_CH_LOADED reads ch [n][F] in the storage dtype;
 * XL_CH_MIDPOINT_POWERS forms channel c of sample i as m_i^c (m the interval
 * midpoint; channels 1, m, m^2 give the depth moments), with no channel
 * gradient.  Samples, offsets and streams as for the colour path; errors:
 * XL_EINVAL for NULL arrays, bad dtype or source, F outside 1..8, P outside
 * 0..4 or a pair index outside [0, F); XL_EHIP if a launch fails.
 */
#define XL_CH_LOADED 0
#define XL_CH_MIDPOINT_POWERS 1
#define XL_BREAKABLE_MAX_CH 8
#define XL_BREAKABLE_MAX_PAIRS 4

typedef struct xl_breakable {
  int32_t dtype;        /* storage of sigma, loaded channels and their gradients */
  int32_t source;       /* XL_CH_LOADED or XL_CH_MIDPOINT_POWERS */
  int32_t n_ch;         /* F, 1..XL_BREAKABLE_MAX_CH */
  int32_t n_pairs;      /* P, 0..XL_BREAKABLE_MAX_PAIRS */
  int32_t pair_a[XL_BREAKABLE_MAX_PAIRS]; /* channel a_p of second-order member p */
  int32_t pair_b[XL_BREAKABLE_MAX_PAIRS]; /* channel b_p (the inner integral's) */
  const void* sigma;    /* device [n] */
  const void* ch;       /* device [n][F] (XL_CH_LOADED), else unused */
  const float* t_start; /* device [n] */
  const float* t_end;   /* device [n] */
  int64_t n;
} xl_breakable;

/* Per segment: seg_out float32 [1+F+P][n_seg] = (tau, Phi, Psi), written. */
int xl_render_breakable_fwd(const xl_breakable* b, const int64_t* seg_offsets, int64_t n_seg,
                            float* seg_out, void* stream);
/* Per ray: ray_out float32 [1+F+P][n_rays] = (T, Phi, Psi), folding the
 * segments listed by ray_offsets / seg_ids front to back (a ray without
 * segments gets (1, 0, ..., 0); ids outside [0, n_seg) are skipped).  Only the
 * channel count, pairs and dtype of `b` are used. */
int xl_merge_breakable_fwd(const xl_breakable* b, const float* seg_out, int64_t n_seg,
                           const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                           float* ray_out, void* stream);
/* Backward of the merge: grad_ray = dl/d(T, Phi, Psi) [1+F+P][n_rays] ->
 * grad_seg = dl/d(tau, Phi, Psi) [1+F+P][n_seg] of every listed segment
 * (overwritten there; each segment listed by at most one ray). */
int xl_merge_breakable_bwd(const xl_breakable* b, const float* seg_out, int64_t n_seg,
                           const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                           const float* grad_ray, float* grad_seg, void* stream);
/* Backward of the segments: from seg_out (the forward's) and grad_seg, writes
 * dl/dsigma [n] (added to grad_sigma's contents when accumulate_sigma != 0)
 * and, for XL_CH_LOADED, dl/dch [n][F] (grad_ch may be NULL otherwise).
 * Per-sample suffix sums are a forward total minus an inclusive prefix: their
 * rounding error is absolute, about one float32 ulp of that total. */
int xl_render_breakable_bwd(const xl_breakable* b, const int64_t* seg_offsets, int64_t n_seg,
                            const float* seg_out, const float* grad_seg, void* grad_sigma,
                            void* grad_ch, int32_t accumulate_sigma, void* stream);

/*
 * Render server: continuous batching of novel-view requests (the inference
 * path of App. A.2: per-region composite, then the merge on one device).
 * Requests are generated on the device (stand-in for per-region NeRF
 * evaluation), rendered with xl_render_segments_fwd + xl_merge_fwd and kept
 * until released.  Up to max_slots requests run at once, each on its own HIP
 * stream.  The server allocates hbm_budget_bytes of device memory once, at
 * creation, and carves every request's buffers out of it.  Slots take
 * requests in arrival order; a slot plans its request's generation (which
 * fixes the exact footprint), then admissions run one at a time: the request
 * waits until that much memory is free next to the requests in flight and
 * the results not yet released.  A request whose footprint exceeds the whole
 * budget fails at once with XL_ENOMEM.  Each slot also holds the generator's
 * plan workspace (about 470 bytes per ray of its largest request so far),
 * allocated outside the budget when a larger request first arrives.  Results hold their memory until xl_serve_release: a client
 * that keeps results while it waits for later requests must leave room for
 * them.  A request's result does not depend on the others.  All functions
 * are thread-safe.
 */
typedef struct xl_server xl_server;

typedef struct xl_serve_config {
  uint64_t hbm_budget_bytes; /* device memory allocated at creation for requests */
  int32_t max_slots;         /* requests processed concurrently (>= 1) */
  int32_t max_queue;         /* requests waiting for a slot; XL_EAGAIN beyond */
  int32_t device;            /* HIP device ordinal */
  int32_t dtype;             /* sample storage: XL_F32, XL_BF16, XL_F16, XL_BF16_F16 */
  int32_t merge_fp64;        /* 1: merge with XL_MERGE_FP64 */
  int32_t reserved;
} xl_serve_config;

typedef struct xl_request {
  int32_t width, height;     /* one ray per pixel */
  int32_t grid[3];           /* regions of the scene */
  int32_t n_min, n_max;      /* samples per ray */
  int32_t inject_fault;      /* tests: fail this request with XL_EFAULT */
  double sigma_mu, sigma_s, zero_frac;
  double width_mean, t_far;  /* 0 = defaults 0.02 and 3 */
  uint64_t seed;             /* the view's generator seed */
} xl_request;

typedef struct xl_result {
  int32_t status;            /* XL_OK, XL_PENDING or an error code */
  int32_t reserved;
  const float* ray_out;      /* device [7][n_rays], valid until xl_serve_release */
  int64_t n_rays, n_samples, n_segments;
  uint64_t footprint_bytes;  /* HBM the request held while rendering */
  int64_t latency_us;        /* completion - arrival (host monotonic clock) */
  int64_t queue_us;          /* admission to a slot - arrival */
  int64_t device_us;         /* generation + composite + merge on the device */
  int64_t device_start_us;   /* its device interval, from one origin per server */
  int64_t device_end_us;     /* (-1 if unavailable): intervals of requests compare */
} xl_result;

typedef struct xl_serve_stats {
  int64_t completed, failed, queued, samples;
  uint64_t budget_used_bytes;
  int64_t p50_latency_us, p99_latency_us, max_latency_us;
  int64_t span_us;           /* first arrival to last completion */
} xl_serve_stats;

/* XL_ENOMEM if the budget cannot be allocated, XL_EINVAL for bad settings. */
int xl_serve_create(const xl_serve_config* cfg, xl_server** out);
/* Non-blocking; XL_EAGAIN when max_queue requests are already waiting. */
int xl_serve_submit(xl_server* s, const xl_request* req, uint64_t* ticket);
/* Waits up to timeout_us (0: no wait, < 0: forever).  Returns XL_PENDING, or
 * the request's final status (XL_OK or its error) with *out filled in. */
int xl_serve_poll(xl_server* s, uint64_t ticket, xl_result* out, int64_t timeout_us);
/* Copies a finished request's ray tuple [7][n_rays] to dst (device), async on
 * `stream`; a later xl_serve_release waits for the copy. */
int xl_serve_copy_result(xl_server* s, uint64_t ticket, float* dst, void* stream);
/* Returns a finished request's result to the server's memory once copies made
 * by xl_serve_copy_result have completed (ray_out becomes invalid). */
int xl_serve_release(xl_server* s, uint64_t ticket);
int xl_serve_stats_get(xl_server* s, xl_serve_stats* out);
/* Stops the server: requests not yet admitted fail with XL_EAGAIN, requests
 * already rendering complete; then every result and buffer is freed.  No other
 * call on the server may overlap this one or follow it. */
int xl_serve_destroy(xl_server* s);

#ifdef __cplusplus
}
#endif

#endif /* XL_H */
