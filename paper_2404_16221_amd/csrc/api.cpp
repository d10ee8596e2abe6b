// C ABI of libxl: argument validation, error reporting and dispatch to the
// HIP launchers.  Nothing here allocates on the compute path.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int ok() {
  g_err[0] = '\0';
  return XL_OK;
}

int hip_status(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(XL_EHIP, "%s: %s", what, hipGetErrorString(e));
  return ok();
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_samples(const xl_samples* s, xl::SamplesDev* out) {
  if (s == nullptr) return fail(XL_EINVAL, "samples descriptor is NULL");
  if (s->dtype != XL_F32 && s->dtype != XL_BF16 && s->dtype != XL_F16 && s->dtype != XL_BF16_F16)
    return fail(XL_EINVAL, "unknown sample dtype %d", s->dtype);
  if (s->n < 0) return fail(XL_EINVAL, "negative sample count %lld", (long long)s->n);
  if (s->n > 0) {
    if (!s->sigma || !s->rgb || !s->t_start || !s->t_end)
      return fail(XL_EINVAL, "NULL sample array with n = %lld", (long long)s->n);
    if (!aligned16(s->sigma) || !aligned16(s->rgb) || !aligned16(s->t_start) ||
        !aligned16(s->t_end))
      return fail(XL_EINVAL, "sample arrays must be 16-byte aligned");
  }
  out->dtype = s->dtype;
  out->sigma = s->sigma;
  out->rgb = s->rgb;
  out->t0 = s->t_start;
  out->t1 = s->t_end;
  out->n = s->n;
  return XL_OK;
}

int check_segments(const xl::SamplesDev& s, const int64_t* seg_offsets, int64_t n_seg) {
  if (n_seg < 0) return fail(XL_EINVAL, "negative segment count %lld", (long long)n_seg);
  if (seg_offsets == nullptr) return fail(XL_EINVAL, "seg_offsets is NULL");
  if (n_seg == 0 && s.n > 0) return fail(XL_EINVAL, "%lld samples but no segments", (long long)s.n);
  return XL_OK;
}

}  // namespace

namespace xl {
int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}
int clear_error() { return ok(); }
}  // namespace xl

extern "C" {

int xl_version(void) { return 100; }

const char* xl_last_error(void) { return g_err; }

size_t xl_segments_workspace_bytes(int64_t n) {
  return xl::segments_workspace_bytes(n > 0 ? n : 0);
}

int xl_render_segments_fwd(const xl_samples* s, const int64_t* seg_offsets, int64_t n_seg,
                           float* seg_out, void* workspace, size_t workspace_bytes,
                           void* stream) {
  xl::SamplesDev d;
  int rc = check_samples(s, &d);
  if (rc) return rc;
  if ((rc = check_segments(d, seg_offsets, n_seg))) return rc;
  if (n_seg > 0 && seg_out == nullptr) return fail(XL_EINVAL, "seg_out is NULL");
  if (!aligned16(seg_out)) return fail(XL_EINVAL, "seg_out must be 16-byte aligned");
  if (d.n > 0) {
    if (workspace == nullptr) return fail(XL_EINVAL, "workspace is NULL");
    if (!aligned16(workspace)) return fail(XL_EINVAL, "workspace must be 16-byte aligned");
    if (workspace_bytes < xl_segments_workspace_bytes(d.n))
      return fail(XL_EINVAL, "workspace too small: %zu < %zu bytes", workspace_bytes,
                  xl_segments_workspace_bytes(d.n));
  }
  return hip_status(xl::launch_segments_fwd(d, seg_offsets, n_seg, seg_out,
                                            workspace,
                                            static_cast<hipStream_t>(stream)),
                    "xl_render_segments_fwd launch");
}

int xl_render_segments_fwd_static(const xl_samples* s, const int64_t* seg_offsets,
                                  int64_t n_seg, float* seg_out, void* stream) {
  xl::SamplesDev d;
  int rc = check_samples(s, &d);
  if (rc) return rc;
  if ((rc = check_segments(d, seg_offsets, n_seg))) return rc;
  if (n_seg > 0 && seg_out == nullptr) return fail(XL_EINVAL, "seg_out is NULL");
  if (!aligned16(seg_out)) return fail(XL_EINVAL, "seg_out must be 16-byte aligned");
  const size_t need = xl_segments_workspace_bytes(d.n);
  if (need > static_cast<size_t>(XL_STATIC_SCRATCH_BYTES))
    return fail(XL_EINVAL,
                "%lld samples need %zu bytes of tile records, more than the static scratch "
                "holds (%zu bytes); use xl_render_segments_fwd with a workspace",
                static_cast<long long>(d.n), need, static_cast<size_t>(XL_STATIC_SCRATCH_BYTES));
  void* ws = nullptr;
  if (d.n > 0 && n_seg > 0) {
    rc = hip_status(xl::static_scratch(&ws), "xl_render_segments_fwd_static scratch address");
    if (rc) return rc;
  }
  return hip_status(xl::launch_segments_fwd(d, seg_offsets, n_seg, seg_out, ws,
                                            static_cast<hipStream_t>(stream)),
                    "xl_render_segments_fwd_static launch");
}

int xl_render_segments_bwd(const xl_samples* s, const int64_t* seg_offsets, int64_t n_seg,
                           const void* workspace, size_t workspace_bytes, const float* grad_seg,
                           void* grad_sigma, void* grad_rgb, void* stream) {
  xl::SamplesDev d;
  int rc = check_samples(s, &d);
  if (rc) return rc;
  if ((rc = check_segments(d, seg_offsets, n_seg))) return rc;
  if (d.n > 0) {
    if (workspace == nullptr || grad_seg == nullptr || grad_sigma == nullptr || grad_rgb == nullptr)
      return fail(XL_EINVAL, "NULL workspace or gradient array");
    if (!aligned16(workspace) || !aligned16(grad_seg) || !aligned16(grad_sigma) || !aligned16(grad_rgb))
      return fail(XL_EINVAL, "workspace and gradient arrays must be 16-byte aligned");
    if (workspace_bytes < xl_segments_workspace_bytes(d.n))
      return fail(XL_EINVAL, "workspace too small: %zu < %zu bytes", workspace_bytes,
                  xl_segments_workspace_bytes(d.n));
  }
  return hip_status(xl::launch_segments_bwd(d, seg_offsets, n_seg,
                                            workspace, grad_seg,
                                            grad_sigma, grad_rgb, static_cast<hipStream_t>(stream)),
                    "xl_render_segments_bwd launch");
}

static int check_merge_args(const float* seg_out, int64_t n_seg, const int64_t* region_offsets,
                            int32_t n_regions, const int64_t* ray_offsets, const int64_t* seg_ids,
                            int64_t n_rays, int32_t flags) {
  if (n_seg < 0 || n_rays < 0) return fail(XL_EINVAL, "negative count");
  if (flags & ~(XL_MERGE_FP64 | XL_MERGE_STAGED))
    return fail(XL_EINVAL, "unknown merge flags 0x%x", flags);
  if (n_rays > 0 && ray_offsets == nullptr) return fail(XL_EINVAL, "ray_offsets is NULL");
  if (n_seg > 0 && (seg_out == nullptr || seg_ids == nullptr))
    return fail(XL_EINVAL, "seg_out or seg_ids is NULL");
  if (!aligned16(seg_out)) return fail(XL_EINVAL, "seg_out must be 16-byte aligned");
  if (region_offsets != nullptr && n_regions < 1)
    return fail(XL_EINVAL, "n_regions %d with region_offsets given", n_regions);
  return XL_OK;
}

int xl_merge_fwd(const float* seg_out, int64_t n_seg, const int64_t* region_offsets,
                 int32_t n_regions, const int64_t* ray_offsets, const int64_t* seg_ids,
                 int64_t n_rays, float* ray_out, int32_t flags, void* stream) {
  int rc = check_merge_args(seg_out, n_seg, region_offsets, n_regions, ray_offsets, seg_ids,
                            n_rays, flags);
  if (rc) return rc;
  if (n_rays > 0 && ray_out == nullptr) return fail(XL_EINVAL, "ray_out is NULL");
  return hip_status(xl::launch_merge_fwd(seg_out, n_seg, region_offsets, n_regions, ray_offsets,
                                         seg_ids, n_rays, ray_out, (flags & XL_MERGE_FP64) != 0,
                                         (flags & XL_MERGE_STAGED) != 0,
                                         static_cast<hipStream_t>(stream)),
                    "xl_merge_fwd launch");
}

int xl_merge_bwd(const float* seg_out, int64_t n_seg, const int64_t* region_offsets,
                 int32_t n_regions, const int64_t* ray_offsets, const int64_t* seg_ids,
                 int64_t n_rays, const float* grad_ray, float* grad_seg, int32_t flags,
                 void* stream) {
  int rc = check_merge_args(seg_out, n_seg, region_offsets, n_regions, ray_offsets, seg_ids,
                            n_rays, flags);
  if (rc) return rc;
  if (n_rays > 0 && (grad_ray == nullptr || (n_seg > 0 && grad_seg == nullptr)))
    return fail(XL_EINVAL, "grad_ray or grad_seg is NULL");
  if (!aligned16(grad_seg)) return fail(XL_EINVAL, "grad_seg must be 16-byte aligned");
  return hip_status(xl::launch_merge_bwd(seg_out, n_seg, region_offsets, n_regions, ray_offsets,
                                         seg_ids, n_rays, grad_ray, grad_seg,
                                         (flags & XL_MERGE_FP64) != 0,
                                         (flags & XL_MERGE_STAGED) != 0,
                                         static_cast<hipStream_t>(stream)),
                    "xl_merge_bwd launch");
}

int xl_check_inputs(const xl_samples* s, const int64_t* seg_offsets, int64_t n_seg,
                    const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                    void* stream) {
  xl::SamplesDev d;
  int rc = check_samples(s, &d);
  if (rc) return rc;
  if ((rc = check_segments(d, seg_offsets, n_seg))) return rc;
  if (n_rays < 0) return fail(XL_EINVAL, "negative ray count");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int* code = nullptr;
  hipError_t e = hipMalloc(&code, sizeof(int));
  if (e != hipSuccess) return fail(XL_ENOMEM, "hipMalloc: %s", hipGetErrorString(e));
  const int big = 1 << 30;
  e = hipMemcpyAsync(code, &big, sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = xl::launch_check(d, seg_offsets, n_seg, ray_offsets, seg_ids, n_rays, code, st);
  int host = big;
  if (e == hipSuccess) e = hipMemcpyAsync(&host, code, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const hipError_t ef = hipFree(code);
  if (e == hipSuccess) e = ef;
  if (e != hipSuccess) return fail(XL_EHIP, "xl_check_inputs: %s", hipGetErrorString(e));
  static const char* what[] = {"",
                               "seg_offsets[0] != 0",
                               "seg_offsets[n_seg] != n",
                               "seg_offsets decreasing",
                               "t_end < t_start",
                               "intervals unsorted or overlapping inside a segment",
                               "ray_offsets must run from 0 to n_seg",
                               "ray_offsets decreasing",
                               "seg_ids out of range"};
  if (host != big && host >= 1 && host <= 8) return fail(XL_EINVAL, "invalid input: %s", what[host]);
  return ok();
}

static int check_gen(const xl_gen_params* p) {
  if (p == nullptr) return fail(XL_EINVAL, "generator parameters are NULL");
  if (p->n_rays < 0 || p->ray0 < 0) return fail(XL_EINVAL, "negative ray count or offset");
  if (p->n_min < 0 || p->n_max < p->n_min) return fail(XL_EINVAL, "bad samples-per-ray range");
  for (int c = 0; c < 3; ++c)
    if (p->grid[c] < 1) return fail(XL_EINVAL, "grid dimensions must be >= 1");
  if (static_cast<int64_t>(p->grid[0]) * p->grid[1] * p->grid[2] > 256 ||
      p->grid[0] + p->grid[1] + p->grid[2] > 18)
    return fail(XL_EINVAL, "grid too large (at most 256 regions, gx + gy + gz <= 18)");
  if (!(p->width_mean > 0) || !(p->t_far > 0)) return fail(XL_EINVAL, "bad width_mean or t_far");
  return XL_OK;
}

size_t xl_gen_workspace_bytes(const xl_gen_params* p) {
  return check_gen(p) == XL_OK ? xl::gen_workspace_bytes(p) : 0;
}

int xl_gen_plan(const xl_gen_params* p, void* workspace, size_t workspace_bytes,
                int64_t* n_samples, int64_t* n_seg, void* stream) {
  int rc = check_gen(p);
  if (rc) return rc;
  if (!workspace || workspace_bytes < xl::gen_workspace_bytes(p) || !n_samples || !n_seg)
    return fail(XL_EINVAL, "workspace missing or too small, or NULL outputs");
  int overflow = 0;
  rc = hip_status(xl::gen_plan(p, workspace, static_cast<hipStream_t>(stream), n_samples, n_seg,
                               &overflow),
                  "xl_gen_plan");
  if (rc) return rc;
  if (overflow) return fail(XL_EINVAL, "a ray crossed more regions than the grid allows");
  return ok();
}

int xl_gen_fill(const xl_gen_params* p, int32_t dtype, void* workspace, size_t workspace_bytes,
                int64_t n_seg, void* sigma, void* rgb, float* t_start, float* t_end,
                int64_t* seg_offsets, int64_t* ray_offsets, int64_t* seg_ids,
                int64_t* region_offsets, void* stream) {
  int rc = check_gen(p);
  if (rc) return rc;
  if (dtype != XL_F32 && dtype != XL_BF16 && dtype != XL_F16 && dtype != XL_BF16_F16)
    return fail(XL_EINVAL, "unknown sample dtype %d", dtype);
  if (!workspace || workspace_bytes < xl::gen_workspace_bytes(p))
    return fail(XL_EINVAL, "workspace missing or too small");
  if (n_seg < 0) return fail(XL_EINVAL, "negative segment count");
  if (p->n_rays > 0 && (!sigma || !rgb || !t_start || !t_end))
    return fail(XL_EINVAL, "NULL sample array");
  return hip_status(xl::gen_fill(p, dtype, workspace, n_seg, sigma, rgb, t_start, t_end, seg_offsets,
                                 ray_offsets, seg_ids, region_offsets,
                                 static_cast<hipStream_t>(stream)),
                    "xl_gen_fill");
}

int xl_partition_build(const float* points, int64_t n_points, int32_t levels, int32_t* axis,
                       float* plane) {
  if (levels < 0 || levels > 6) return fail(XL_EINVAL, "levels must be in [0, 6], got %d", levels);
  if (n_points < 0) return fail(XL_EINVAL, "negative point count");
  if (n_points > 0 && points == nullptr) return fail(XL_EINVAL, "points is NULL");
  if (levels > 0 && (axis == nullptr || plane == nullptr))
    return fail(XL_EINVAL, "axis or plane is NULL");
  if (xl::partition_build(points, n_points, levels, axis, plane) != XL_OK)
    return fail(XL_EINVAL, "points must be finite");
  return ok();
}

static int check_pack(const xl_rays* rays, const int32_t* axis, const float* plane, int32_t levels,
                      void* workspace, size_t workspace_bytes) {
  if (rays == nullptr) return fail(XL_EINVAL, "rays descriptor is NULL");
  if (levels < 0 || levels > 6) return fail(XL_EINVAL, "levels must be in [0, 6], got %d", levels);
  if (rays->n_rays < 0) return fail(XL_EINVAL, "negative ray count");
  if (rays->ray_offsets == nullptr) return fail(XL_EINVAL, "ray_offsets is NULL");
  if (rays->n_rays > 0 && (!rays->origins || !rays->dirs || !rays->t_start || !rays->t_end))
    return fail(XL_EINVAL, "NULL ray or sample array");
  if (levels > 0 && (axis == nullptr || plane == nullptr))
    return fail(XL_EINVAL, "axis or plane is NULL");
  if (workspace == nullptr || workspace_bytes < xl::pack_workspace_bytes(rays->n_rays, levels))
    return fail(XL_EINVAL, "workspace missing or too small (%zu < %zu bytes)", workspace_bytes,
                xl::pack_workspace_bytes(rays->n_rays, levels));
  return XL_OK;
}

size_t xl_pack_workspace_bytes(int64_t n_rays, int32_t levels) {
  if (n_rays < 0 || levels < 0 || levels > 6) return 0;
  return xl::pack_workspace_bytes(n_rays, levels);
}

int xl_pack_plan(const xl_rays* rays, const int32_t* axis, const float* plane, int32_t levels,
                 void* workspace, size_t workspace_bytes, int64_t* n_pieces, int64_t* n_seg,
                 void* stream) {
  int rc = check_pack(rays, axis, plane, levels, workspace, workspace_bytes);
  if (rc) return rc;
  if (!n_pieces || !n_seg) return fail(XL_EINVAL, "NULL outputs");
  return hip_status(xl::pack_plan(rays, axis, plane, levels, workspace,
                                  static_cast<hipStream_t>(stream), n_pieces, n_seg),
                    "xl_pack_plan");
}

int xl_pack_fill(const xl_rays* rays, const int32_t* axis, const float* plane, int32_t levels,
                 void* workspace, size_t workspace_bytes, int64_t n_seg, float* t_start,
                 float* t_end, int64_t* src, int64_t* seg_offsets, int64_t* ray_offsets,
                 int64_t* seg_ids, int32_t* seg_box, int64_t* region_offsets, void* stream) {
  int rc = check_pack(rays, axis, plane, levels, workspace, workspace_bytes);
  if (rc) return rc;
  if (n_seg < 0) return fail(XL_EINVAL, "negative segment count");
  if (!seg_offsets || !ray_offsets || (n_seg > 0 && (!t_start || !t_end || !seg_ids)))
    return fail(XL_EINVAL, "NULL output array");
  return hip_status(xl::pack_fill(rays, axis, plane, levels, workspace, n_seg, t_start, t_end, src,
                                  seg_offsets, ray_offsets, seg_ids, seg_box, region_offsets,
                                  static_cast<hipStream_t>(stream)),
                    "xl_pack_fill");
}

static int check_features(const xl_features* f, const int64_t* seg_offsets, int64_t n_seg) {
  if (f == nullptr) return fail(XL_EINVAL, "features descriptor is NULL");
  if (f->dtype != XL_F32 && f->dtype != XL_BF16 && f->dtype != XL_F16)
    return fail(XL_EINVAL, "unknown sample dtype %d", f->dtype);
  if (f->n_feat != 4 && f->n_feat != 8 && f->n_feat != 16 && f->n_feat != 32)
    return fail(XL_EINVAL, "n_feat must be 4, 8, 16 or 32, got %d", f->n_feat);
  if (f->n < 0 || n_seg < 0) return fail(XL_EINVAL, "negative count");
  if (f->n > 0 && (!f->sigma || !f->feat || !f->t_start || !f->t_end))
    return fail(XL_EINVAL, "NULL sample array with n = %lld", (long long)f->n);
  if (f->n > 0 && !aligned16(f->feat)) return fail(XL_EINVAL, "feat must be 16-byte aligned");
  if (seg_offsets == nullptr) return fail(XL_EINVAL, "seg_offsets is NULL");
  if (n_seg == 0 && f->n > 0) return fail(XL_EINVAL, "%lld samples but no segments", (long long)f->n);
  return XL_OK;
}

int xl_render_features_fwd(const xl_features* f, const int64_t* seg_offsets, int64_t n_seg,
                           float* phi_seg, float* tau_seg, void* stream) {
  int rc = check_features(f, seg_offsets, n_seg);
  if (rc) return rc;
  if (n_seg > 0 && phi_seg == nullptr) return fail(XL_EINVAL, "phi_seg is NULL");
  return hip_status(xl::launch_features_fwd(f, seg_offsets, n_seg, phi_seg, tau_seg,
                                            static_cast<hipStream_t>(stream)),
                    "xl_render_features_fwd launch");
}

int xl_render_features_bwd(const xl_features* f, const int64_t* seg_offsets, int64_t n_seg,
                           const float* phi_seg, const float* grad_phi_seg,
                           const float* grad_tau_seg, void* grad_sigma, void* grad_feat,
                           int32_t accumulate_sigma, void* stream) {
  int rc = check_features(f, seg_offsets, n_seg);
  if (rc) return rc;
  if (n_seg > 0 && (!phi_seg || !grad_phi_seg))
    return fail(XL_EINVAL, "phi_seg or grad_phi_seg is NULL");
  if (f->n > 0 && (!grad_sigma || !grad_feat)) return fail(XL_EINVAL, "NULL gradient array");
  if (f->n > 0 && !aligned16(grad_feat)) return fail(XL_EINVAL, "grad_feat must be 16-byte aligned");
  return hip_status(xl::launch_features_bwd(f, seg_offsets, n_seg, phi_seg, grad_phi_seg, grad_tau_seg,
                                            grad_sigma, grad_feat, accumulate_sigma != 0,
                                            static_cast<hipStream_t>(stream)),
                    "xl_render_features_bwd launch");
}

static int check_feature_merge(const float* tau_seg, const float* phi_seg, int32_t n_feat, int64_t n_seg,
                               const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays) {
  if (n_feat != 4 && n_feat != 8 && n_feat != 16 && n_feat != 32)
    return fail(XL_EINVAL, "n_feat must be 4, 8, 16 or 32, got %d", n_feat);
  if (n_seg < 0 || n_rays < 0) return fail(XL_EINVAL, "negative count");
  if (n_rays > 0 && ray_offsets == nullptr) return fail(XL_EINVAL, "ray_offsets is NULL");
  if (n_seg > 0 && (!tau_seg || !phi_seg || !seg_ids))
    return fail(XL_EINVAL, "tau_seg, phi_seg or seg_ids is NULL");
  return XL_OK;
}

int xl_merge_features_fwd(const float* tau_seg, const float* phi_seg, int32_t n_feat, int64_t n_seg,
                          const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                          float* phi_ray, void* stream) {
  int rc = check_feature_merge(tau_seg, phi_seg, n_feat, n_seg, ray_offsets, seg_ids, n_rays);
  if (rc) return rc;
  if (n_rays > 0 && phi_ray == nullptr) return fail(XL_EINVAL, "phi_ray is NULL");
  return hip_status(xl::launch_features_merge(tau_seg, phi_seg, n_feat, n_seg, ray_offsets, seg_ids,
                                              n_rays, phi_ray, static_cast<hipStream_t>(stream)),
                    "xl_merge_features_fwd launch");
}

int xl_merge_features_bwd(const float* tau_seg, const float* phi_seg, int32_t n_feat, int64_t n_seg,
                          const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                          const float* grad_ray, float* grad_phi_seg, float* grad_tau_seg,
                          void* stream) {
  int rc = check_feature_merge(tau_seg, phi_seg, n_feat, n_seg, ray_offsets, seg_ids, n_rays);
  if (rc) return rc;
  if (n_rays > 0 && (!grad_ray || (n_seg > 0 && (!grad_phi_seg || !grad_tau_seg))))
    return fail(XL_EINVAL, "grad_ray, grad_phi_seg or grad_tau_seg is NULL");
  return hip_status(xl::launch_features_merge_bwd(tau_seg, phi_seg, n_feat, n_seg, ray_offsets, seg_ids,
                                                  n_rays, grad_ray, grad_phi_seg, grad_tau_seg,
                                                  static_cast<hipStream_t>(stream)),
                    "xl_merge_features_bwd launch");
}

// ---------------------------------------------------------------- breakable integrals
static int check_breakable_shape(const xl_breakable* b) {
  if (b == nullptr) return fail(XL_EINVAL, "breakable descriptor is NULL");
  if (b->dtype != XL_F32 && b->dtype != XL_BF16 && b->dtype != XL_F16)
    return fail(XL_EINVAL, "unknown sample dtype %d", b->dtype);
  if (b->source != XL_CH_LOADED && b->source != XL_CH_MIDPOINT_POWERS)
    return fail(XL_EINVAL, "unknown channel source %d", b->source);
  if (b->n_ch < 1 || b->n_ch > XL_BREAKABLE_MAX_CH)
    return fail(XL_EINVAL, "n_ch must be 1..%d, got %d", XL_BREAKABLE_MAX_CH, b->n_ch);
  if (b->n_pairs < 0 || b->n_pairs > XL_BREAKABLE_MAX_PAIRS)
    return fail(XL_EINVAL, "n_pairs must be 0..%d, got %d", XL_BREAKABLE_MAX_PAIRS, b->n_pairs);
  for (int p = 0; p < b->n_pairs; ++p)
    if (b->pair_a[p] < 0 || b->pair_a[p] >= b->n_ch || b->pair_b[p] < 0 || b->pair_b[p] >= b->n_ch)
      return fail(XL_EINVAL, "pair %d (%d, %d) names a channel outside [0, %d)", p, b->pair_a[p],
                  b->pair_b[p], b->n_ch);
  return XL_OK;
}

static int check_breakable(const xl_breakable* b, const int64_t* seg_offsets, int64_t n_seg) {
  int rc = check_breakable_shape(b);
  if (rc) return rc;
  if (b->n < 0 || n_seg < 0) return fail(XL_EINVAL, "negative count");
  if (b->n > 0 && (!b->sigma || !b->t_start || !b->t_end))
    return fail(XL_EINVAL, "NULL sample array with n = %lld", (long long)b->n);
  if (b->n > 0 && b->source == XL_CH_LOADED && !b->ch) return fail(XL_EINVAL, "ch is NULL");
  if (seg_offsets == nullptr) return fail(XL_EINVAL, "seg_offsets is NULL");
  if (n_seg == 0 && b->n > 0) return fail(XL_EINVAL, "%lld samples but no segments", (long long)b->n);
  return XL_OK;
}

int xl_render_breakable_fwd(const xl_breakable* b, const int64_t* seg_offsets, int64_t n_seg,
                            float* seg_out, void* stream) {
  int rc = check_breakable(b, seg_offsets, n_seg);
  if (rc) return rc;
  if (n_seg > 0 && seg_out == nullptr) return fail(XL_EINVAL, "seg_out is NULL");
  return hip_status(xl::launch_breakable_fwd(b, seg_offsets, n_seg, seg_out,
                                             static_cast<hipStream_t>(stream)),
                    "xl_render_breakable_fwd launch");
}

int xl_render_breakable_bwd(const xl_breakable* b, const int64_t* seg_offsets, int64_t n_seg,
                            const float* seg_out, const float* grad_seg, void* grad_sigma,
                            void* grad_ch, int32_t accumulate_sigma, void* stream) {
  int rc = check_breakable(b, seg_offsets, n_seg);
  if (rc) return rc;
  if (n_seg > 0 && (!seg_out || !grad_seg)) return fail(XL_EINVAL, "seg_out or grad_seg is NULL");
  if (b->n > 0 && !grad_sigma) return fail(XL_EINVAL, "grad_sigma is NULL");
  if (b->n > 0 && b->source == XL_CH_LOADED && !grad_ch) return fail(XL_EINVAL, "grad_ch is NULL");
  return hip_status(xl::launch_breakable_bwd(b, seg_offsets, n_seg, seg_out, grad_seg, grad_sigma,
                                             grad_ch, accumulate_sigma != 0,
                                             static_cast<hipStream_t>(stream)),
                    "xl_render_breakable_bwd launch");
}

static int check_breakable_merge(const xl_breakable* b, const float* seg_out, int64_t n_seg,
                                 const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays) {
  int rc = check_breakable_shape(b);
  if (rc) return rc;
  if (n_seg < 0 || n_rays < 0) return fail(XL_EINVAL, "negative count");
  if (n_rays > 0 && ray_offsets == nullptr) return fail(XL_EINVAL, "ray_offsets is NULL");
  if (n_seg > 0 && (!seg_out || !seg_ids)) return fail(XL_EINVAL, "seg_out or seg_ids is NULL");
  return XL_OK;
}

int xl_merge_breakable_fwd(const xl_breakable* b, const float* seg_out, int64_t n_seg,
                           const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                           float* ray_out, void* stream) {
  int rc = check_breakable_merge(b, seg_out, n_seg, ray_offsets, seg_ids, n_rays);
  if (rc) return rc;
  if (n_rays > 0 && ray_out == nullptr) return fail(XL_EINVAL, "ray_out is NULL");
  return hip_status(xl::launch_breakable_merge(b, seg_out, n_seg, ray_offsets, seg_ids, n_rays,
                                               ray_out, static_cast<hipStream_t>(stream)),
                    "xl_merge_breakable_fwd launch");
}

int xl_merge_breakable_bwd(const xl_breakable* b, const float* seg_out, int64_t n_seg,
                           const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                           const float* grad_ray, float* grad_seg, void* stream) {
  int rc = check_breakable_merge(b, seg_out, n_seg, ray_offsets, seg_ids, n_rays);
  if (rc) return rc;
  if (n_rays > 0 && (!grad_ray || (n_seg > 0 && !grad_seg)))
    return fail(XL_EINVAL, "grad_ray or grad_seg is NULL");
  return hip_status(xl::launch_breakable_merge_bwd(b, seg_out, n_seg, ray_offsets, seg_ids, n_rays,
                                                   grad_ray, grad_seg,
                                                   static_cast<hipStream_t>(stream)),
                    "xl_merge_breakable_bwd launch");
}

}  // extern "C"
