// Internal launcher interface between the C ABI (api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/xl.h"

namespace xl {

struct SamplesDev {
  int dtype;
  const void* sigma;
  const void* rgb;
  const float* t0;
  const float* t1;
  int64_t n;
};


int64_t num_tiles(int64_t n);
size_t segments_workspace_bytes(int64_t n);  // per-tile records

hipError_t launch_segments_fwd(const SamplesDev& s, const int64_t* seg_offsets, int64_t n_seg,
                               float* seg_out, void* workspace, hipStream_t stream);
// Device address of this GPU's static tile-record scratch
// (XL_STATIC_SCRATCH_BYTES), looked up once per device.
hipError_t static_scratch(void** ptr);
hipError_t launch_segments_bwd(const SamplesDev& s, const int64_t* seg_offsets, int64_t n_seg,
                               const void* workspace, const float* grad_seg, void* grad_sigma,
                               void* grad_rgb, hipStream_t stream);
// region_offsets (n_regions + 1 entries) may be NULL: then the tuples are
// gathered per ray; otherwise staged per workgroup through LDS from 4M
// segments up, or at any size with `staged` (merge.hip).
hipError_t launch_merge_fwd(const float* seg_out, int64_t n_seg, const int64_t* region_offsets,
                            int n_regions, const int64_t* ray_offsets, const int64_t* seg_ids,
                            int64_t n_rays, float* ray_out, bool fp64, bool staged,
                            hipStream_t stream);
hipError_t launch_merge_bwd(const float* seg_out, int64_t n_seg, const int64_t* region_offsets,
                            int n_regions, const int64_t* ray_offsets, const int64_t* seg_ids,
                            int64_t n_rays, const float* grad_ray, float* grad_seg, bool fp64,
                            bool staged, hipStream_t stream);
// Device-side input checks; writes the number of the first failed check (0 =
// none) to *code_dev.
hipError_t launch_check(const SamplesDev& s, const int64_t* seg_offsets, int64_t n_seg,
                        const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                        int* code_dev, hipStream_t stream);

// Thread-local error message for xl_last_error (api.cpp); returns `code`.
int set_error(int code, const char* fmt, ...);
int clear_error();

// Device generator (gen.hip).
size_t gen_workspace_bytes(const xl_gen_params* p);
int64_t gen_max_segments(const xl_gen_params* p);  // rays x regions a ray can cross
hipError_t gen_plan(const xl_gen_params* p, void* ws, hipStream_t st, int64_t* n_samples,
                    int64_t* n_seg, int* overflow, int64_t* pinned = nullptr);
hipError_t gen_fill(const xl_gen_params* p, int dtype, void* ws, int64_t n_seg, void* sigma,
                    void* rgb, float* t_start, float* t_end, int64_t* seg_offsets,
                    int64_t* ray_offsets, int64_t* seg_ids, int64_t* region_offsets,
                    hipStream_t st);

// Exclusive scan of int64 (gen.hip): out[0..n] with out[n] = total; tmp holds
// scan_tmp_elems(n) entries.
size_t scan_tmp_elems(int64_t n);
hipError_t scan_exclusive(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, size_t tmp_elems,
                          hipStream_t st);

// Spatial partitioning (partition.cpp, host) and sample distribution (pack.hip).
int partition_build(const float* points, int64_t n, int levels, int32_t* axis, float* plane);
size_t pack_workspace_bytes(int64_t n_rays, int levels);
hipError_t pack_plan(const xl_rays* rays, const int32_t* axis, const float* plane, int levels,
                     void* ws, hipStream_t st, int64_t* n_pieces, int64_t* n_seg);
hipError_t pack_fill(const xl_rays* rays, const int32_t* axis, const float* plane, int levels,
                     void* ws, int64_t n_seg, float* t_start, float* t_end, int64_t* src,
                     int64_t* seg_offsets, int64_t* ray_offsets, int64_t* seg_ids, int32_t* seg_box,
                     int64_t* region_offsets, hipStream_t st);

// Feature channels (features.hip).
hipError_t launch_features_fwd(const xl_features* f, const int64_t* seg_offsets, int64_t n_seg,
                               float* phi_seg, float* tau_seg, hipStream_t st);
hipError_t launch_features_bwd(const xl_features* f, const int64_t* seg_offsets, int64_t n_seg,
                               const float* phi_seg, const float* grad_phi_seg, const float* grad_tau_seg,
                               void* grad_sigma, void* grad_feat, int accumulate, hipStream_t st);
hipError_t launch_features_merge(const float* tau_seg, const float* phi_seg, int F, int64_t n_seg,
                                 const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                                 float* phi_ray, hipStream_t st);
hipError_t launch_features_merge_bwd(const float* tau_seg, const float* phi_seg, int F, int64_t n_seg,
                                     const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                                     const float* grad_ray, float* grad_phi_seg, float* grad_tau_seg,
                                     hipStream_t st);

// Breakable integrals (breakable.hip).
hipError_t launch_breakable_fwd(const xl_breakable* b, const int64_t* seg_offsets, int64_t n_seg,
                                float* seg_out, hipStream_t st);
hipError_t launch_breakable_bwd(const xl_breakable* b, const int64_t* seg_offsets, int64_t n_seg,
                                const float* seg_out, const float* grad_seg, void* grad_sigma,
                                void* grad_ch, int accumulate, hipStream_t st);
hipError_t launch_breakable_merge(const xl_breakable* b, const float* seg_out, int64_t n_seg,
                                  const int64_t* ray_offsets, const int64_t* seg_ids, int64_t n_rays,
                                  float* ray_out, hipStream_t st);
hipError_t launch_breakable_merge_bwd(const xl_breakable* b, const float* seg_out, int64_t n_seg,
                                      const int64_t* ray_offsets, const int64_t* seg_ids,
                                      int64_t n_rays, const float* grad_ray, float* grad_seg,
                                      hipStream_t st);

}  // namespace xl
