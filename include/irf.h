/*
 * irf -- irradiance field with visibility on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the per-frame probe update and the probe query of the method of
 * Majercik, Marrs, Spjut and McGuire, "Scaling Probe-Based Real-Time Dynamic
 * Global Illumination for Production" (JCGT 2021, arXiv 2009.10796), which
 * refines DDGI (Majercik et al. 2019).  Sections of the paper are cited by
 * title.
 *
 * Conventions
 *  - Every call returns irf_status; IRF_OK is 0.  Arguments are validated
 *    before anything is launched.  A failed call leaves the context unchanged
 *    and sets a thread-local message (irf_last_error).
 *  - Host pointers are read during the call only (copied).  Device pointers
 *    belong to the caller; the library never frees them and reads/writes
 *    them asynchronously on the given stream, so they must stay alive until
 *    that stream's work is done.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Vectors are float32 x,y,z triples; matrices are row-major float32.
 *  - Triangles are counter-clockwise seen from their front side.
 *  - Probe q of a volume with counts (nx, ny, nz) has grid index (i, j, k),
 *    q = i + nx * (j + ny * k), and sits at origin + (i, j, k) * spacing plus
 *    its offset.
 *  - One context per thread; a context is tied to the HIP device it was
 *    created on.
 */
#ifndef IRF_H
#define IRF_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IRF_OK = 0,
  IRF_E_INVALID = 1,     /* bad argument (NULL, out of range, non-finite, ...) */
  IRF_E_NOMEM = 2,       /* device or host allocation failed */
  IRF_E_HIP = 3,         /* a HIP runtime call failed (message has details) */
  IRF_E_STATE = 4,       /* call not valid now (e.g. update before bind) */
  IRF_E_UNSUPPORTED = 5  /* valid request the library does not implement */
} irf_status;

/* Probe states (Section "Probe States"). */
enum {
  IRF_OFF = 0, IRF_SLEEPING = 1, IRF_NEWLY_AWAKE = 2, IRF_NEWLY_VIGILANT = 3,
  IRF_AWAKE = 4, IRF_VIGILANT = 5
};

/* Atlas storage types and blend arithmetic. */
enum { IRF_ATLAS_F32 = 0, IRF_ATLAS_F16 = 1 };
enum { IRF_BLEND_F32 = 0, IRF_BLEND_BF16 = 1, IRF_BLEND_F16 = 2, IRF_BLEND_F32_VALU = 3 };

#define IRF_MAX_VOLUMES 8
#define IRF_MAX_LIGHTS 32
#define IRF_MAX_ROTATIONS 8

typedef struct irf_ctx irf_ctx;

/* Error reporting.  The message is thread-local and valid until the next
   failing call on this thread. */
const char* irf_status_str(irf_status s);
const char* irf_last_error(void);
/* Library version, e.g. "irf 0.1 gfx950". */
const char* irf_version(void);

/* Context: owns the scene (BVH), light set, per-frame scratch and the
   volume descriptions.  `hip_device` is a HIP device ordinal. */
irf_status irf_create(int32_t hip_device, irf_ctx** out);
/* Frees every library-owned device allocation.  NULL is accepted. */
void irf_destroy(irf_ctx* ctx);

/* Triangle scene.  Host arrays; copied.  The BVH is built on the host
   (binned SAH, two-wide, depth-limited) and uploaded synchronously.  A later
   call replaces the scene.
     vertices      [n_vertices][3]
     indices       [n_triangles][3], each < n_vertices
     tri_material  [n_triangles], each < n_materials
     tri_object    [n_triangles], 0 = static, k > 0 = dynamic object k; NULL
                   means all static (classification rays see static triangles
                   only; dynamic objects wake nearby probes, Section "Full
                   Probe Initialization Algorithm")
     albedo, emission [n_materials][3] (Lambertian albedo; emitted radiance)
     specular         [n_materials][3] mirror reflectance for the
                   second-order glossy pass, or NULL (zero) */
typedef struct {
  const float* vertices;
  int64_t n_vertices;
  const uint32_t* indices;
  int64_t n_triangles;
  const uint32_t* tri_material;
  const uint32_t* tri_object;
  const float* albedo;
  const float* emission;
  int32_t n_materials;
  const float* specular;
} irf_scene_desc;
irf_status irf_set_scene(irf_ctx* ctx, const irf_scene_desc* desc);

/* Lights used by hit shading (Section "Probe Update": hits are shaded by the
   deferred-shading model, here Lambertian with shadow rays).  Host arrays,
   copied into the context; the next launched frame uses them, so a capture of
   irf_update_probes records the lights current at capture time.
     dir_to_light   [n_dir][3] unit vectors toward each directional light
     dir_irradiance [n_dir][3] irradiance on a surface facing the light
     point_pos      [n_point][3]
     point_intensity[n_point][3] radiant intensity, W/sr
     sky[3]         radiance returned by rays that hit nothing
   n_dir + n_point <= IRF_MAX_LIGHTS. */
typedef struct {
  const float* dir_to_light;
  const float* dir_irradiance;
  int32_t n_dir;
  const float* point_pos;
  const float* point_intensity;
  int32_t n_point;
  float sky[3];
} irf_lights_desc;
irf_status irf_set_lights(irf_ctx* ctx, const irf_lights_desc* desc);

/* Probe volume.  Volumes are blended from the first created (densest) to the
   last (sparsest) (Section "Multiple Probe Volumes").
     counts          >= 2 per axis
     rays_per_probe  multiple of 32, 32..1024 (spherical Fibonacci rays under
                     one random rotation per frame, Section "Probe Update")
     hysteresis_*    in [0, 1]: weight of the old texel (Eq. U)
     cos_power       exponent p of the distance weight max(0, n.w)^p, > 0
     self_shadow_bias B of Eq. 1, >= 0
     max_distance    distance clamp for misses and hits; <= 0 selects
                     1.5 * |spacing|
     cheb_power      exponent of the Chebyshev visibility weight, 1..4
     atlas_dtype     IRF_ATLAS_F32 or IRF_ATLAS_F16
     blend           how the texels are blended (Eq. U): IRF_BLEND_F32,
                     IRF_BLEND_BF16, IRF_BLEND_F16 = one shared (texel x ray)
                     weight matrix times the rays of the probes on the matrix
                     cores, inputs in that precision, float32 accumulation and
                     float32 normalisation by the sum of the stored weights;
                     IRF_BLEND_F32_VALU = vector ALU, one workgroup per probe
                     with its rays in LDS (the paper's compute-shader shape)
     irradiance_gamma perception encoding of irradiance texels (Section
                     "Perception-based exponential encoding"): texels store
                     the new mean to the power 1/gamma and blend in that
                     encoding; the query raises each probe's sample to
                     gamma/2, blends, and squares.  0 or 1 = linear texels;
                     else in [1, 16] (the paper uses 5)
     texel_thresholds 1 = per-texel irradiance hysteresis (Section "Fast
                     Convergence Heuristics"): a texel whose largest
                     per-channel change in stored units exceeds 0.25 blends
                     with hysteresis lowered by 0.15 (not below 0), above 0.8
                     with hysteresis 0; distance texels are not affected
     tracking        1 = a window that follows the camera (Section "Tracking
                     Windows"; counts >= 5 per axis): moved with
                     irf_track_volume, stored as a circular buffer, and
                     blended with a camera-centred weight (the per-axis ramp
                     tightened by one cell, Section "Multiple Probe Volumes");
                     the camera starts at the window centre */
typedef struct {
  float origin[3];
  float spacing[3];
  int32_t counts[3];
  int32_t rays_per_probe;
  float hysteresis_irr;
  float hysteresis_dist;
  float cos_power;
  float self_shadow_bias;
  float max_distance;
  int32_t cheb_power;
  int32_t atlas_dtype;
  int32_t blend;
  float irradiance_gamma;
  int32_t texel_thresholds;
  int32_t tracking;
} irf_volume_desc;
irf_status irf_create_volume(irf_ctx* ctx, const irf_volume_desc* desc, int32_t* volume_id);

/* Sizes in bytes of the caller-owned buffers of a volume, and its probe
   count.  Layouts:
     irradiance [P][8][8][4]  (RGB + unused 4th channel; float or half)
     distance   [P][16][16][2] (mean distance, mean distance^2)
     states     [P] uint8
     offsets    [P][3] float  */
typedef struct {
  int64_t n_probes;
  int64_t irradiance_bytes;
  int64_t distance_bytes;
  int64_t states_bytes;
  int64_t offsets_bytes;
} irf_buffer_sizes;
irf_status irf_volume_sizes(const irf_ctx* ctx, int32_t volume, irf_buffer_sizes* out);

/* Binds caller-owned device buffers (16-byte aligned) to a volume.  The
   update reads and writes irradiance, distance and states in place; offsets
   may be NULL (all zero; irf_optimize_probes then refuses), and are written
   only by irf_optimize_probes.  Initial contents are the caller's (zeros and
   IRF_NEWLY_VIGILANT, or the result of irf_classify). */
irf_status irf_bind_volume(irf_ctx* ctx, int32_t volume, void* irradiance, void* distance,
                           uint8_t* states, const float* offsets);

/* Probe classification (Section "Full Probe Initialization Algorithm", steps
   1-2): per probe, K x rays_per_probe distance-only rays against static
   triangles under the K host rotations [K][9] (1 <= K <= IRF_MAX_ROTATIONS).
   More than 25 % backfaces -> OFF; else a front face closer than the largest
   spacing -> NEWLY_VIGILANT; else SLEEPING; then sleeping probes inside the
   box of a dynamic object grown by one cell plus the self-shadow bias become
   NEWLY_AWAKE.  Writes the bound states of every volume.  Async. */
irf_status irf_classify(irf_ctx* ctx, const float* rotations, int32_t K, void* stream);

/* Tracking window (Section "Tracking Windows") of a volume created with
   tracking = 1.  Along each axis, while the camera (host float[3]) is more
   than one spacing from the window centre, the window moves one cell toward
   it: the plane left behind is reused, in place, for the plane entering in
   front (circular buffer; the storage slot of logical probe i is
   (i + phase) mod n, see irf_volume_window).  Entering probes start over:
   their texels and offsets are zeroed and they are classified as in
   irf_classify with the K host rotations [K][9].  The camera is kept for the
   blend weight of queries.  shift (host int32[3], may be NULL) receives the
   cells moved.  Moving the window changes the volume's origin and phase, so
   a captured frame graph must be captured again.  Async. */
irf_status irf_track_volume(irf_ctx* ctx, int32_t volume, const float* camera, const float* rotations, int32_t K,
                            int32_t* shift, void* stream);
/* Current window of a volume: origin of logical probe (0,0,0), storage
   phase per axis, camera position of the blend weight. */
irf_status irf_volume_window(const irf_ctx* ctx, int32_t volume, float origin[3], int32_t phase[3], float camera[3]);

/* Probe relocation (Section "Probe Position Adjustment"), run before
   irf_classify: `iterations` passes (the paper uses 5), pass i tracing every
   probe's rays against static triangles from its current position under
   host rotation rotations[i][9].  A probe seeing more than 25 % backfaces
   moves along the vector to its closest backface, scaled as far as the
   offset limit allows less 1e-3 of the scale, if that scale exceeds 1 (it
   gets through); otherwise, unless its farthest and closest front faces lie
   within 60 degrees, it steps min(0.2, distance) toward the farthest front
   face, if that stays within the limit; else it keeps its offset.
   offset_limit in (0, 0.5] is a fraction of the spacing per axis.  Reads and
   writes the bound offsets of every volume (IRF_E_STATE if a volume has
   none).  Async. */
irf_status irf_optimize_probes(irf_ctx* ctx, const float* rotations, int32_t iterations, float offset_limit,
                               void* stream);

/* One update frame for all bound volumes (Section "Probe Update"): state
   step (dynamic-object wake/sleep), compaction of active probes (Newly
   Awake, Newly Vigilant, Awake, Vigilant), spherical-Fibonacci rays under
   `rotation` (host [9]), nearest-hit BVH traversal, hit shading (direct
   light with shadow rays, emission, previous frame's irradiance queried from
   all volumes, backface rule), blend of irradiance (cosine weights) and mean
   distance / distance^2 (cosine^p weights) with hysteresis (0 for Newly
   states), border texels, promotion of Newly states.  Async. */
irf_status irf_update_probes(irf_ctx* ctx, const float* rotation, void* stream);

/* The same frame for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   it calls no hipMalloc, hipFree or other allocating routine.  Its frame
   scratch (parameters, active list, ray directions, weight rows, hit
   records, shadow-task queues, visibility bytes, ray radiance) is carved
   from one static device array of IRF_NOALLOC_SCRATCH_BYTES that each GPU
   the library runs on holds until the process ends, shared by every
   context and call on that GPU; it keeps the last call's contents (each
   frame writes what it reads).  Calls that overlap on one GPU (two streams,
   two threads) race on it: order them.  A frame whose scratch (the sizes
   irf_update_probes would allocate for the bound volumes and lights) exceeds
   the array, or a differentiable context (irf_set_differentiable), returns
   IRF_E_UNSUPPORTED before any launch.  Results (atlases, states) are those
   of irf_update_probes bit for bit; the frame's rays run in index order
   (the per-volume coherent trace order is a library allocation), and
   irf_ray_records / irf_frame_stats do not see this frame (IRF_E_STATE until
   the next irf_update_probes).  Async. */
#define IRF_NOALLOC_SCRATCH_BYTES (128ll << 20)
irf_status irf_update_probes_noalloc(irf_ctx* ctx, const float* rotation, void* stream);

/* The same frame, with its atlas writes (the blend) ordered after
   `atlas_event` (a hipEvent_t the caller recorded, typically after the
   previous frame's queries on another stream; NULL: none).  Everything
   before the blend -- state step, rays, traversal, shadow rays, hit shading,
   which only read the atlases -- may then run beside those queries: an
   engine's probe trace for the next frame overlapping its shading of the
   current one.  When the scene has dynamic objects the state step can put
   Awake probes to sleep, which changes what a query samples, so then the
   whole frame is ordered after the event.  The caller orders its next queries after this frame (an
   event recorded on `stream` after this call).  IRF_E_HIP if waiting on the
   event fails.  Async. */
irf_status irf_update_probes_after(irf_ctx* ctx, const float* rotation, void* stream, void* atlas_event);

/* Query E(X, n, w_o) (Section "Probe Query", Eq. 1, Section "Multiple Probe
   Volumes") for n points.  pos, nrm, view, out_rgb: device [n][3] float;
   view is the unit direction from the point toward the viewer.  The result
   is in the units of the irradiance texels (cosine-weighted mean radiance).
   n = 0 is a no-op.  Async. */
irf_status irf_query_irradiance(irf_ctx* ctx, const float* pos, const float* nrm, const float* view,
                                int64_t n, float* out_rgb, void* stream);

/* One update frame (irf_update_probes) that also answers n irradiance
   queries (irf_query_irradiance: same arrays, layouts and units) against the
   atlases and probe states as they stood before this frame, i.e. the result
   of the previous frame.  `out_rgb` receives exactly what
   irf_query_irradiance on the same stream just before irf_update_probes
   would have written, and the frame's results are those of
   irf_update_probes; only the schedule differs.  The queries run inside the
   frame's probe-ray trace and shadow-ray launches, split by the tuning's
   query_shadow (neither launch writes an atlas or a probe state): the
   traversals' waves wait on dependent node fetches and leave issue slots
   that the queries' arithmetic fills (Section "Probe Query" for what a
   query computes, Section "Probe Update" for the frame).
   A renderer that shades frame f with the probes of update f issues
   update f+1 together with the queries of frame f.  When the scene has
   dynamic objects the frame's state step can rewrite the states a query
   reads, so the queries then run first, as their own launch.  n = 0 is a
   plain frame; n < 0, a NULL rotation or (with n > 0) a NULL array:
   IRF_E_INVALID before any launch.  Async. */
irf_status irf_update_probes_query(irf_ctx* ctx, const float* rotation, const float* pos, const float* nrm,
                                   const float* view, int64_t n, float* out_rgb, void* stream);

/* Launch shapes of the frame's main kernels: the number of workgroups of
   the persistent probe-ray traversal, shadow-ray traversal, hit shading and
   matrix-core blend; each strides over the work of all volumes.  With the
   shadow rays in batches (shadow_refill = 0) the hit shading's indirect
   term (the previous frame's irradiance at each hit, which needs the hit
   alone) runs in the shadow-ray launch, on shade_blocks workgroups of its
   own, and the shading launch adds the direct light.  0 selects
   one workgroup per work unit of the largest possible frame.  A new context
   starts at 0 except for the shadow rays: 16 workgroups per compute unit,
   what stays resident at once at eight waves per SIMD, each lane looping
   over the frame's tasks, instead of a workgroup for every shadow ray the
   largest frame could queue (most of them empty).  shadow_refill selects
   how the shadow rays are spread over lanes: 0 in batches of 64 tasks (a
   wave moves on when the longest ray of its batch ends); n in [1, 64] a
   fixed range of tasks per wave whose lanes take the range's next task
   whenever at least n of them are idle.  blend_rsplit is the blend's tile
   shape: how many workgroups share one block of 8 probes (1, 2 or 4; 0
   selects 4), each taking 16 / rsplit of the 16 row tiles of the weight
   matrix, so the block's rays are staged rsplit times and each wave
   multiplies 4 / rsplit row tiles.  query_shadow splits the query batch of
   irf_update_probes_query: per mille of its points answered in the
   shadow-ray launch (batched shadow rays only; with shadow_refill > 0, or
   no lights, all of them run in the probe-ray trace launch), the rest in
   the trace launch (a new context: 500).  Results do not depend on any of
   these.  The launch shapes are normally chosen by the autotuner
   (paper_2009_10796_amd/autotune.py).  IRF_E_INVALID for negative values,
   shadow_refill above 64, blend_rsplit not in {0, 1, 2, 4} or query_shadow
   above 1000. */
typedef struct {
  int32_t trace_blocks;
  int32_t shadow_blocks;
  int32_t shade_blocks;
  int32_t blend_blocks;
  int32_t shadow_refill;
  int32_t blend_rsplit;
  int32_t query_shadow;
} irf_tuning;
irf_status irf_set_tuning(irf_ctx* ctx, const irf_tuning* tuning);
irf_status irf_get_tuning(const irf_ctx* ctx, irf_tuning* tuning);

/* A whole update frame captured as a HIP graph.  irf_graph_capture records
   the frame's launches on `stream` (not the null stream) without running
   them; irf_graph_launch replays it with a new rotation and the context's
   current lights (the frame's parameters are the argument block of its
   frame-start node, updated before each launch).  A graph stays valid while the scene,
   volumes, bound buffers, light count, dynamic objects and tuning are
   unchanged; otherwise irf_graph_launch returns IRF_E_STATE and the frame
   must be captured again. */
typedef struct irf_graph irf_graph;
irf_status irf_graph_capture(irf_ctx* ctx, void* stream, irf_graph** out);
/* The frame of irf_update_probes_query captured the same way: each
   irf_graph_launch of it is an update frame that also answers the n queries
   at the device arrays given here (pos, nrm, view, out_rgb: [n][3] float,
   fixed at capture; the caller may rewrite their contents between launches)
   against the atlases and states the previous frame left.  Same errors as
   irf_graph_capture, and IRF_E_INVALID for n < 0 or (n > 0) a NULL array. */
irf_status irf_graph_capture_query(irf_ctx* ctx, void* stream, const float* pos, const float* nrm,
                                   const float* view, int64_t n, float* out_rgb, irf_graph** out);
irf_status irf_graph_launch(irf_ctx* ctx, irf_graph* graph, const float* rotation, void* stream);
void irf_graph_destroy(irf_graph* graph);

/* ---- adjoint (differentiation of query -> blend -> hit shading with the
   ray hits and shadow decisions of the forward frame held fixed) ----
   Gradients are float32 device buffers with the atlas layouts
   (irradiance [P][8][8][4], distance [P][16][16][2]) and accumulate (+=);
   per-volume buffers are passed as a host array of n_volumes device
   pointers.  Volumes must have float32 atlases, linear irradiance texels
   (irradiance_gamma 0 or 1) and no per-texel thresholds
   (IRF_E_UNSUPPORTED otherwise). */

/* While enabled, each irf_update_probes also saves the frame's input atlases
   and its states after the state step (library memory), for
   irf_update_backward. */
irf_status irf_set_differentiable(irf_ctx* ctx, int32_t enable);
/* Replaces the materials' emitted radiance from a device array [n_materials][3]. */
irf_status irf_set_emission(irf_ctx* ctx, const float* emission, void* stream);
/* dLoss/d(atlases) of irf_query_irradiance at the same points given
   grad_out = dLoss/dE [n][3] (device); reads the current atlases.  Adds
   (+=) into grad_irr[v] / grad_dist[v] (device, the layout of the volume's
   atlases).  Each texel's terms are summed in point order without atomics,
   so the result is the same bit for bit from call to call; the terms go
   through library memory (about 0.25 GB, allocated on the first call) in
   batches of 2^22 / (8 x volumes) points. */
irf_status irf_query_backward(irf_ctx* ctx, const float* pos, const float* nrm, const float* view, int64_t n,
                              const float* grad_out, float* const* grad_irr, float* const* grad_dist, void* stream);
/* Backward of the last update frame: from dLoss/d(output atlases) to
   dLoss/d(input atlases) and dLoss/d(emission) [n_materials][3], all added
   (+=) into the caller's device arrays.  The blend is differentiated with
   float32 weights whatever the forward blend mode.  Gradients are summed in
   a fixed order (texels: ray order; emitters: ray order per material), so
   they are the same bit for bit from call to call.  Reads the frame's ray
   count back to the host (synchronizes `stream`). */
irf_status irf_update_backward(irf_ctx* ctx, float* const* grad_new_irr, float* const* grad_new_dist,
                               float* const* grad_prev_irr, float* const* grad_prev_dist, float* grad_emission,
                               void* stream);

/* Per-ray records of the last update for one volume, in active-probe order
   (ascending probe index) then ray order.  Synchronizes `stream`.  Writes at
   most `capacity` records to the device buffer `out` and the count to
   *count (host). */
typedef struct {
  int32_t tri;    /* original triangle index, -1 for a miss */
  float t;        /* hit distance (unclamped), +inf for a miss */
  float rgb[3];   /* shaded radiance carried by the ray */
  float d;        /* distance entered into the distance texels */
  uint32_t vis;   /* bit l: shadow ray toward light l (directional first) unblocked */
  int32_t probe;  /* probe index within the volume */
} irf_ray_record;
irf_status irf_ray_records(irf_ctx* ctx, int32_t volume, irf_ray_record* out, int64_t capacity,
                           int64_t* count, void* stream);

/* Second-order glossy (Section "Second Order Glossy"): for n surface points
   (device float[n][3] positions, unit normals, unit directions toward the
   viewer) the radiance arriving along each point's mirror direction,
   out_rgb (device float[n][3]).  The mirror ray starts from the point lifted
   off its surface by 1e-4 max(1, |X|inf); a miss sees the sky, a backface
   is black; a front hit Y (material m, geometric normal ng) is shaded as a
   probe-ray hit -- emission + albedo * (direct light / pi + the probes'
   irradiance at Y) -- plus specular[m] times the probes' filtered radiance
   in Y's own mirror direction (the query at Y with the texels sampled in
   that direction), so second and later glossy bounces come from the
   probes.  records (device, n entries, or NULL) receives per point the hit
   triangle, distance, radiance and shadow visibility (d = 0, probe = -1).
   n = 0 is valid.  Async. */
irf_status irf_trace_glossy(irf_ctx* ctx, const float* pos, const float* nrm, const float* view, int64_t n,
                            float* out_rgb, irf_ray_record* records, void* stream);


/* Frame statistics of the last update (synchronizes `stream`):
   out[0] active probes, out[1] probe rays traced, out[2] shadow rays traced,
   out[3] probe rays that hit a front face. */
irf_status irf_frame_stats(irf_ctx* ctx, int64_t out[4], void* stream);

/* Traversal work of the last update, re-traced in a counting mode that is
   never part of a frame (synchronizes `stream`): out[0] BVH nodes fetched
   and out[1] triangles tested by the probe rays, out[2] nodes and out[3]
   triangles by the shadow rays.  A node is 64 bytes, a triangle 48. */
irf_status irf_traversal_stats(irf_ctx* ctx, int64_t out[4], void* stream);

/* Kernel timing.  While enabled, every kernel the library launches is
   bracketed by HIP events recorded on the stream it is launched on;
   irf_profile_read synchronizes those events and returns, per kernel name,
   the number of launches and their summed duration (ms) since the last
   reset.  Costs one event pair per launch; off by default. */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
} irf_kernel_time;
irf_status irf_profile_enable(irf_ctx* ctx, int32_t enable);
irf_status irf_profile_read(irf_ctx* ctx, irf_kernel_time* out, int32_t capacity, int32_t* count, int32_t reset);

/* Host-side helpers that need no device (used by tests of the host logic). */
/* Validates a volume description exactly as irf_create_volume does. */
irf_status irf_validate_volume_desc(const irf_volume_desc* desc);
/* Builds the BVH of a scene on the host and reports its statistics:
   out[0] nodes, out[1] leaves, out[2] max depth, out[3] SAH cost,
   out[4] 1 if every triangle is referenced exactly once and every node box
   contains its children, else 0. */
irf_status irf_bvh_stats(const irf_scene_desc* desc, double out[5]);

#ifdef __cplusplus
}
#endif
#endif
