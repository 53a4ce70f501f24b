// Internal types of the irf library (device-visible structures and launch
// entry points shared between translation units).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <vector>

#include "../../include/irf.h"

namespace irf {

// Kernel timing: while the API times a stage it points g_kernel_timing at a
// start/stop event pair; irf_launch then stamps the first kernel's start and
// every kernel's end on the dispatch itself (hipExtLaunchKernel), so the
// measured time is kernel execution only.
struct KernelTiming {
  hipEvent_t start, stop;
  bool first;
};
extern thread_local KernelTiming* g_kernel_timing;

template <typename F, typename... Args>
inline void irf_launch(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, Args... args) {
  KernelTiming* t = g_kernel_timing;
  if (!t) {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
    return;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, t->first ? t->start : nullptr, t->stop, 0u, args...);
  t->first = false;
}


constexpr int kIrrTile = 8;      // 6x6 interior + one-texel border
constexpr int kDistTile = 16;    // 14x14 interior + one-texel border
constexpr int kIrrTexels = kIrrTile * kIrrTile;
constexpr int kDistTexels = kDistTile * kDistTile;
constexpr int kMaxDepth = 48;    // BVH depth limit = traversal stack size
constexpr int kLeafMax = 8;

// Device view of one probe volume.
struct VolumeGPU {
  float origin[3];
  float spacing[3];
  float inv_spacing[3];     // 1 / spacing, correctly rounded float32 (grid coordinates by a product)
  int32_t counts[3];
  int32_t n_probes;
  int32_t rays;
  float alpha_irr, alpha_dist;
  float cos_power;
  int32_t cos_power_int;    // p if p is an integer in [1, 64], else 0
  float bias;               // B of the self-shadow bias
  float dmax;
  int32_t cheb_power;
  int32_t atlas_f16;
  int32_t blend;
  float gamma, inv_gamma, half_gamma;   // perception encoding of irradiance texels (1 = linear)
  int32_t thresholds;       // per-texel irradiance hysteresis thresholds (0 / 1)
  int32_t phase[3];         // tracking window: slot of logical probe i is (i + phase) mod n
  int32_t tracking;         // 1: camera-centred blend weight
  float camera[3];          // camera position for that weight
  int32_t probe_base;       // first global probe id of this volume
  int32_t omega_base;       // first entry of this volume in the direction table
  int64_t weight_base;      // byte offset of this volume's blend weights
  void* irr;                // [P][8][8] float4 or half4
  void* dist;               // [P][16][16] float2 or half2
  uint8_t* states;          // [P]
  const float* offsets;     // [P][3] or null
  const int16_t* order;     // [rays] order in which the probe-ray traversal takes a probe's rays
};

struct VolumeSet {
  VolumeGPU v[IRF_MAX_VOLUMES];
  int32_t n;
};

// Lights by value (kernel argument).
struct LightSet {
  float dir[IRF_MAX_LIGHTS][3];     // directional: unit vector toward the light
  float irr[IRF_MAX_LIGHTS][3];     // directional: irradiance; point: intensity
  float pos[IRF_MAX_LIGHTS][3];     // point: position
  int32_t n_dir;
  int32_t n_point;
  float sky[3];
};

// Per-frame parameters read by the frame's kernels from device memory.
struct FrameParams {
  float R[9];      // rotation of the spherical-Fibonacci pattern
  LightSet L;
};

// Launch shapes chosen by the autotuner (0 = default).
struct Tuning {
  int32_t trace_blocks;
  int32_t shadow_blocks;
  int32_t shade_blocks;
  int32_t blend_blocks;
  int32_t shadow_refill;   // 0: shadow rays in batches of 64; n > 0: lane refill at n idle lanes
  int32_t blend_rsplit;    // workgroups per probe block of the blend: 1, 2 or 4 (0: 4)
  int32_t query_shadow;    // irf_update_probes_query: per mille of its batch answered in the shadow launch
};

// Dynamic-object boxes (state step and classification wake rule).
struct ObjectBoxes {
  const float* lo;   // [n][3]
  const float* hi;   // [n][3]
  int32_t n;
};

// Shadow tasks are queued in kTaskRegions regions of the task array, a
// source wave's region chosen by its index, so that waves reserving their
// runs at the same time add to different counters (one shared counter
// serialises every wave of the trace on one address).  One region per lane
// of a wave.
constexpr int kTaskRegions = 64;

// Tasks one region can hold: its share of the source waves of 64 rays, up
// to 64 * n_lights tasks each.
__host__ __device__ inline int64_t task_region_cap(int64_t max_rays, int n_lights) {
  const int64_t waves = (max_rays + 63) / 64;
  return (waves + kTaskRegions - 1) / kTaskRegions * 64 * (int64_t)n_lights;
}

// Per-frame counters written by the compaction kernel.
struct FrameCounters {
  int32_t slot_base[IRF_MAX_VOLUMES + 1];   // active probes of volume v: [slot_base[v], slot_base[v+1])
  int64_t ray_base[IRF_MAX_VOLUMES + 1];    // rays of volume v: [ray_base[v], ray_base[v+1])
  uint64_t task_count[kTaskRegions];        // shadow rays queued in each task region this frame
};

// Scene on the device.
struct SceneGPU {
  const float4* nodes;     // [n_nodes][4]  (two child boxes + child links)
  const float4* tris;      // [n_tris][3]   (v0 | orig id, v1 | object, v2 | material)
  const float4* albedo;    // [M]
  const float4* emission;  // [M]
  const float4* specular;  // [M] mirror reflectance (second-order glossy)
  int32_t n_tris;
  int32_t n_nodes;
  int32_t stack_depth;     // traversal stack entries needed (BVH depth)
};

struct GradSet {
  float* irr[IRF_MAX_VOLUMES];
  float* dist[IRF_MAX_VOLUMES];
};

// Nearest hit of one probe ray.  The hit triangle's geometric normal and
// material ride along, so the hit shading starts without fetching the
// triangle again.
struct HitRec {
  int32_t tri;   // BVH-order triangle, -1 miss
  float t;
  int32_t mat;   // material of the triangle (hits only)
  int32_t pad;
  float n[4];    // unit geometric normal of the triangle in n[0..2] (hits only)
};
static_assert(sizeof(HitRec) == 32, "two 16-byte halves");

// Frame scratch (library-owned device memory).
struct FrameScratch {
  FrameParams* params;      // rotation and lights of the frame
  int32_t* block_active;    // [compaction workgroups] active probes per workgroup
  int32_t* active;          // [max_slots] global probe id per active slot
  FrameCounters* counters;  // device
  float4* omega;            // [sum rays] direction table for this frame
  HitRec* hits;             // [max_rays]
  uint8_t* vis;             // [n_lights][max_rays]
  float4* rays;             // [max_rays] rgb + distance (float32 path)
  float4* shadow_tasks;     // [kTaskRegions][task_region_cap]: one contiguous run per source
                            // wave of 64 rays in its region, light-major; the shadow origin
                            // and, in w, the bits of (ray id << 5 | light)
  float4* grad_rays;        // [max_rays] adjoint: dLoss/d(ray radiance)
  float4* probe_pos;        // [max_slots] position of each active probe this frame (by slot),
                            // w = 1 for a Newly state (blended with no hysteresis), else 0
  void* weights;            // per volume: 256 weight rows x rays (float32 [k][row] or 16-bit [row][k])
  float* inv_row_sum;       // [n_volumes][256] 1 / sum of the stored weights of each row (0 = none)
  int64_t max_rays;
  int32_t max_slots;
};

// ---- host-side BVH builder (bvh_build.cpp)
int build_bvh(const float* vertices, int64_t nv, const uint32_t* indices, int64_t nt,
              const uint32_t* tri_material, const uint32_t* tri_object,
              std::vector<float4>& nodes, std::vector<float4>& tris, double stats[5]);

// ---- launches (kernels_*.hip); all asynchronous on `s`
// Start of an update frame (kernels_frame.hip): the frame's parameters, ray
// directions, matrix-core blend weights and the state step with the active
// list, all in one kernel whose only argument is this struct (a captured
// frame is re-launched with a new rotation by updating that one node).
struct FrameBegin {
  FrameParams p;
  VolumeSet vs;
  ObjectBoxes ob;
  FrameScratch fs;
  int32_t dir_blocks;    // workgroups of ray directions per volume
  int32_t weight_rows;   // workgroups of blend weight rows per volume (0: no matrix-core volume)
  int32_t row_waves;     // waves per weight row (the largest ray count over 64, rounded up)
  int32_t compact;       // 1: the last workgroup steps the states and packs the active list
  int32_t total_probes;  // probes of every volume
};
FrameBegin make_frame_begin(const FrameParams& p, const VolumeSet& vs, ObjectBoxes ob, FrameScratch fs,
                            bool weights);
void launch_frame_begin(const FrameBegin& a, hipStream_t s);
const void* frame_begin_kernel();
void launch_trace(const VolumeSet& vs, SceneGPU sc, FrameScratch fs, int grid, hipStream_t s);
// A batch of irradiance queries (points packed xyz, float32, device memory).
struct QueryBatch {
  const float* pos;
  const float* nrm;
  const float* view;
  float* out;
  int64_t first;   // points [first, first + n) of the arrays
  int64_t n;
};
// The shadow rays in batches of 64 (grid), the indirect term of every
// front-face hit (hit_grid: the hit shading's grid) and a query batch (may be
// empty), one launch.
void launch_shadow_stage(const VolumeSet& vs, SceneGPU sc, int n_lights, FrameScratch fs, int grid, int hit_grid,
                         const QueryBatch& q, hipStream_t s);
// The probe-ray trace with a query batch answered in the same launch.
void launch_trace_query(const VolumeSet& vs, SceneGPU sc, FrameScratch fs, int grid, const QueryBatch& q,
                        hipStream_t s);
// The shadow rays with lane refill (k_shadow_refill, threshold `refill`) and
// the indirect term of every front-face hit (hit_grid), one launch.
void launch_shadow(const VolumeSet& vs, SceneGPU sc, int n_lights, FrameScratch fs, int grid, int hit_grid,
                   int refill, hipStream_t s);
// The hit shading; indirect_done: launch_shadow_stage computed the indirect terms.
void launch_shade(const VolumeSet& vs, SceneGPU sc, FrameScratch fs, int grid, bool indirect_done, hipStream_t s);
void launch_blend(const VolumeSet& vs, FrameScratch fs, hipStream_t s);
void launch_blend_mma(const VolumeSet& vs, FrameScratch fs, int grid, int rsplit, hipStream_t s);
void launch_query(const VolumeSet& vs, const float* pos, const float* nrm, const float* view, int64_t n,
                  float* out, hipStream_t s);
void launch_relocate(const VolumeSet& vs, SceneGPU sc, const float* rotation, float limit, int32_t* back,
                     unsigned long long* keys, hipStream_t s);
// Probes of entering planes of a tracking window: volume `vol` (-1: every
// probe of every volume), logical index in [lo, hi] along some axis.
struct PlaneMask {
  int32_t vol;
  int32_t lo[3], hi[3];
};
void launch_track_reset(const VolumeSet& vs, PlaneMask m, hipStream_t s);
void launch_classify(const VolumeSet& vs, SceneGPU sc, ObjectBoxes boxes, const float* rotations, int K,
                     int32_t* back, uint32_t* tfront, PlaneMask mask, hipStream_t s);
void launch_traversal_stats(const VolumeSet& vs, SceneGPU sc, int n_lights, FrameScratch fs, unsigned long long* out,
                            hipStream_t s);
struct GradSet;
void launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t s);
void launch_set_emission(const float* src, float4* dst, int m, hipStream_t s);
// Scratch of the adjoint's fixed-order gradient sums (library-owned): the
// terms of one batch of query points or rays with their keys (before and
// after the sort) and sorted order, segment bounds and piece offsets over keys
// (probes, then materials), the stored sums of long segments, the blend's
// per-volume normalisers and the sort's temporary storage.
struct AdjointScratch {
  void* terms;             // [max_terms] query terms (40 bytes each)
  uint32_t* keys[2];       // [max_terms] before and after the sort
  uint32_t* idx;           // [max_terms] sorted order (term positions)
  uint32_t* seg_start;     // [max_keys]
  uint32_t* seg_end;       // [max_keys]
  uint32_t* offs;          // [max_keys + 1]
  uint32_t* poffs;         // [max_keys + 1]
  float* partial;          // [max_partial] stored piece sums
  float* norms;            // [volumes][adjoint_norms_per_volume()]
  void* sort_temp;
  size_t sort_bytes;
  int64_t max_terms;
  int64_t max_partial;
};
size_t adjoint_sort_bytes(int64_t max_pairs);
int64_t adjoint_partial_slots(int64_t max_terms);
size_t adjoint_slot_bytes();
int adjoint_norms_per_volume();
hipError_t launch_query_backward(const VolumeSet& vs, const float* pos, const float* nrm, const float* view,
                                 int64_t n, const float* gout, const GradSet& G, const AdjointScratch& A,
                                 hipStream_t s);
hipError_t launch_update_backward(const VolumeSet& prev, SceneGPU sc, FrameScratch fs, const GradSet& Gnew,
                                  const GradSet& Gprev, float* g_emission, int n_materials, int64_t n_rays,
                                  const AdjointScratch& A, hipStream_t s);
void launch_glossy(const VolumeSet& vs, SceneGPU sc, const LightSet& L, const float* pos, const float* nrm,
                   const float* view, int64_t n, float* out, irf_ray_record* rec, hipStream_t s);
void launch_frame_stats(const VolumeSet& vs, SceneGPU sc, FrameScratch fs, unsigned long long* out, hipStream_t s);
void launch_records(const VolumeSet& vs, int vol, SceneGPU sc, FrameScratch fs, int n_lights,
                    irf_ray_record* out, int64_t count, hipStream_t s);

}  // namespace irf
