// Ray traversal and hit shading for the probe update (Section "Probe
// Update": probes trace rotated spherical-Fibonacci rays and shade the hits
// with the deferred-shading model plus the previous frame's probes).
//
// Wavefront layout: one launch traces every active probe ray of every volume
// (their hits are packed across volumes, as the paper packs the ray data of
// all volumes into one texture); one launch traces the shadow rays, ordered
// light-major so that a wave carries 64 neighbouring rays of one probe toward
// one light; one launch shades.  Traversal keeps its stack in LDS, one
// column per lane ([depth][lane] so that lanes at the same depth hit distinct
// banks); nodes are one 64-byte record holding both child boxes.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace irf {

constexpr int kTraceBlock = 128;

struct Ray {
  float3 o, d, inv;
  float3 off_l, off_h;   // slab offsets of the low and high box bounds (see make_ray)
  int kx, ky, kz;
  float Sx, Sy, Sz;
};

__device__ __forceinline__ float sel(float3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// Precomputation of the watertight ray/triangle test (Woop, Benthin and Wald
// 2013): the axis of largest |d| becomes z, the other two are sheared.
__device__ __forceinline__ Ray make_ray(float3 o, float3 d) {
  Ray r;
  r.o = o;
  r.d = d;
  const float tiny = 1e-30f;
  r.inv = f3(1.0f / (fabsf(d.x) > tiny ? d.x : copysignf(tiny, d.x)),
             1.0f / (fabsf(d.y) > tiny ? d.y : copysignf(tiny, d.y)),
             1.0f / (fabsf(d.z) > tiny ? d.z : copysignf(tiny, d.z)));
  // Slab distances as one FMA, t = b * inv + off: off = -o * inv, moved by
  // e = 3u |o * inv| toward the outside of the slab (entry bound earlier,
  // exit bound later), which covers the rounding of -o * inv and of the
  // offset itself; the FMA's own relative rounding is left to the widening
  // of the exit distance in box_hit.
  const float3 oi = f3(r.o.x * r.inv.x, r.o.y * r.inv.y, r.o.z * r.inv.z);
  const float3 e = f3(0x3p-24f * fabsf(oi.x), 0x3p-24f * fabsf(oi.y), 0x3p-24f * fabsf(oi.z));
  // inv > 0: the low bound is the entry; inv < 0: the high bound is
  r.off_l = f3(r.inv.x > 0.0f ? -oi.x - e.x : -oi.x + e.x, r.inv.y > 0.0f ? -oi.y - e.y : -oi.y + e.y,
               r.inv.z > 0.0f ? -oi.z - e.z : -oi.z + e.z);
  r.off_h = f3(r.inv.x > 0.0f ? -oi.x + e.x : -oi.x - e.x, r.inv.y > 0.0f ? -oi.y + e.y : -oi.y - e.y,
               r.inv.z > 0.0f ? -oi.z + e.z : -oi.z - e.z);
  float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  int kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  if (sel(d, kz) < 0.0f) {
    int t = kx;
    kx = ky;
    ky = t;
  }
  r.kx = kx;
  r.ky = ky;
  r.kz = kz;
  float dz = sel(d, kz);
  r.Sx = sel(d, kx) / dz;
  r.Sy = sel(d, ky) / dz;
  r.Sz = 1.0f / dz;
  return r;
}

// Entry distance of the ray into a box within [0, tmax].  Conservative: the
// slab offsets carry the absolute rounding of the origin term, and the exit
// distance is widened by 2 gamma_3 for the relative rounding of the inverse
// direction and the FMA (after Ize 2013), so float rounding never culls a box
// the ray touches.
__device__ __forceinline__ bool box_hit(const Ray& r, float lx, float ly, float lz, float hx, float hy, float hz,
                                        float tmax, float& tnear) {
  float t0x = fmaf(lx, r.inv.x, r.off_l.x), t1x = fmaf(hx, r.inv.x, r.off_h.x);
  float t0y = fmaf(ly, r.inv.y, r.off_l.y), t1y = fmaf(hy, r.inv.y, r.off_h.y);
  float t0z = fmaf(lz, r.inv.z, r.off_l.z), t1z = fmaf(hz, r.inv.z, r.off_h.z);
  float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
  float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
  tnear = tn;
  return tn <= tf * 1.0000004f;
}

// Watertight ray/triangle test; on a hit with 0 < t < tmax returns t.
__device__ __forceinline__ bool tri_hit(const Ray& r, float4 a, float4 b, float4 c, float tmax, float& t) {
  float3 A = f3(a.x - r.o.x, a.y - r.o.y, a.z - r.o.z);
  float3 B = f3(b.x - r.o.x, b.y - r.o.y, b.z - r.o.z);
  float3 C = f3(c.x - r.o.x, c.y - r.o.y, c.z - r.o.z);
  float Akz = sel(A, r.kz), Bkz = sel(B, r.kz), Ckz = sel(C, r.kz);
  float Ax = sel(A, r.kx) - r.Sx * Akz, Ay = sel(A, r.ky) - r.Sy * Akz;
  float Bx = sel(B, r.kx) - r.Sx * Bkz, By = sel(B, r.ky) - r.Sy * Bkz;
  float Cx = sel(C, r.kx) - r.Sx * Ckz, Cy = sel(C, r.ky) - r.Sy * Ckz;
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
  float det = U + V + W;
  if (det == 0.0f) return false;
  float T = U * (r.Sz * Akz) + V * (r.Sz * Bkz) + W * (r.Sz * Ckz);
  if (det > 0.0f) {
    if (!(T > 0.0f) || !(T < tmax * det)) return false;
  } else {
    if (!(T < 0.0f) || !(T > tmax * det)) return false;
  }
  t = T / det;
  return t > 0.0f && t < tmax;
}

__device__ __forceinline__ int bits_i(float f) { return __float_as_int(f); }

// Node value that ends a traversal: negative like a leaf link, and not one
// (a leaf link is ~(first << 3 | count - 1) with first < 2^27).
constexpr int kTraversalDone = INT_MIN;

// Two-wide BVH traversal.  ANY: stop at the first hit (shadow rays).
// STATIC_ONLY: skip triangles of dynamic objects (classification rays).
// `stack` points at this lane's column of the LDS stack; `stride` = block size.
struct NoCount {
  __device__ __forceinline__ void node() {}
  __device__ __forceinline__ void tri() {}
};
struct Count {
  unsigned long long nodes = 0, tris = 0;
  __device__ __forceinline__ void node() { nodes++; }
  __device__ __forceinline__ void tri() { tris++; }
};

template <bool ANY, bool STATIC_ONLY, typename CNT = NoCount>
__device__ inline int traverse(const SceneGPU& sc, const Ray& ray, float tmax, float& t_out, int* stack,
                               int stride, CNT* cnt = nullptr) {
  int best = -1;
  float tbest = tmax;
  if (sc.n_nodes == 0) {
    t_out = tbest;
    return -1;
  }
  int sp = 0;
  int node = 0;
  while (true) {
    while (node >= 0) {
      const float4* np = sc.nodes + (size_t)node * 4;
      float4 n0 = np[0], n1 = np[1], n2 = np[2], n3 = np[3];
      if (cnt) cnt->node();
      float t0, t1;
      const bool h0 = box_hit(ray, n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, tbest, t0);
      const bool h1 = box_hit(ray, n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, tbest, t1);
      const int l0 = bits_i(n3.x), l1 = bits_i(n3.y);
      // branch-free step: descend into the nearer child that was hit and
      // push the other one if both were; with neither, pop.  The slot above
      // the top is always written (it exists: see stack_bytes).
      const bool first0 = h0 & (!h1 | (t0 <= t1));
      const int nearc = first0 ? l0 : l1;
      const int farc = first0 ? l1 : l0;
      const int top = sp < sc.stack_depth - 1 ? sp : sc.stack_depth - 1;
      stack[top * stride] = farc;
      sp = top + ((h0 && h1) ? 1 : 0);
      // the pop is read whether or not it is taken (no branch); an empty
      // stack with no child hit ends the traversal
      const int below = sp > 0 ? sp - 1 : 0;
      const int popped = stack[below * stride];
      const bool any = h0 || h1;
      node = any ? nearc : (sp == 0 ? kTraversalDone : popped);
      sp = any ? sp : below;
    }
    if (node == kTraversalDone) break;
    int code = ~node;
    int first = code >> 3, count = (code & 7) + 1;
    for (int i = first; i < first + count; i++) {
      const float4* tp = sc.tris + (size_t)i * 3;
      float4 a = tp[0], b = tp[1], c = tp[2];
      if (cnt) cnt->tri();
      if (STATIC_ONLY && bits_i(b.w) != 0) continue;
      float t;
      if (tri_hit(ray, a, b, c, tbest, t)) {
        tbest = t;
        best = i;
        if (ANY) {
          t_out = t;
          return i;
        }
      }
    }
    if (sp == 0) break;
    sp--;
    node = stack[sp * stride];
  }
  t_out = tbest;
  return best;
}

// ---- per-ray bookkeeping shared by the update kernels

struct RaySlot {
  int v;       // volume
  int q;       // probe within the volume
  int r;       // ray index within the probe
  int gs;      // slot of the probe in the frame's active list
};

// Ray id -> (volume, probe, ray).  Ray ids of one frame are below 2^27
// (checked by the API), so the division runs in 32 bits.
__device__ __forceinline__ RaySlot locate_ray(const VolumeSet& vs, const FrameCounters& C, const int32_t* active,
                                              int64_t id) {
  int v = 0;
  while (v + 1 < vs.n && id >= C.ray_base[v + 1]) v++;
  const VolumeGPU& V = vs.v[v];
  const uint32_t local = (uint32_t)(id - C.ray_base[v]);
  const uint32_t slot = local / (uint32_t)V.rays;
  RaySlot s;
  s.v = v;
  s.r = (int)(local - slot * (uint32_t)V.rays);
  s.gs = C.slot_base[v] + (int)slot;
  s.q = active[s.gs] - V.probe_base;
  return s;
}

// Position of the ray's probe (computed once per frame at compaction).
__device__ __forceinline__ float3 slot_position(const FrameScratch& fs, const RaySlot& s) {
  const float4 p = fs.probe_pos[s.gs];
  return f3(p.x, p.y, p.z);
}

__device__ __forceinline__ float3 tri_normal(const SceneGPU& sc, int tri) {
  const float4* tp = sc.tris + (size_t)tri * 3;
  float4 a = tp[0], b = tp[1], c = tp[2];
  float3 e1 = f3(b.x - a.x, b.y - a.y, b.z - a.z), e2 = f3(c.x - a.x, c.y - a.y, c.z - a.z);
  return normalize_or_zero(cross(e1, e2));
}

// The normal and the material of a triangle from one fetch of its record.
__device__ __forceinline__ float3 tri_normal_material(const SceneGPU& sc, int tri, int& mat) {
  const float4* tp = sc.tris + (size_t)tri * 3;
  float4 a = tp[0], b = tp[1], c = tp[2];
  mat = bits_i(c.w);
  float3 e1 = f3(b.x - a.x, b.y - a.y, b.z - a.z), e2 = f3(c.x - a.x, c.y - a.y, c.z - a.z);
  return normalize_or_zero(cross(e1, e2));
}

// Shadow-ray origin: the hit lifted off the surface along its normal.
__device__ __forceinline__ float3 shadow_origin(float3 X, float3 ng) {
  float xm = fmaxf(fabsf(X.x), fmaxf(fabsf(X.y), fabsf(X.z)));
  float eps = 1e-4f * fmaxf(1.0f, xm);
  return X + eps * ng;
}

extern __shared__ int dyn_stack[];

__global__ void k_fill_u32(uint32_t* p, uint32_t value, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
// One column of stack_depth entries per lane.  The depth counts the root as 1
// and the leaves, which live in their parent's link, so a lane at an inner
// node of depth k holds at most k - 1 entries and writes at index <= k - 1:
// indices stay below stack_depth - 1, and the spare write of the branch-free
// step (and the clamp in the traversal, which never binds) fits in the
// column.  For the city's depth-20 tree a 128-lane workgroup then takes
// 10 KiB of LDS: sixteen workgroups, eight waves per SIMD.
static inline size_t stack_bytes(const SceneGPU& sc) {
  return sizeof(int) * (size_t)(sc.stack_depth > 0 ? sc.stack_depth : 1) * kTraceBlock;
}

// Whether a shadow ray from front-face hit X toward light l is needed (the
// light is in front of the surface), with its direction and range.
__device__ __forceinline__ bool shadow_ray(const LightSet& L, int l, float3 X, float3 ng, float3& Xs, float3& dl,
                                           float& tmax) {
  Xs = shadow_origin(X, ng);
  if (l < L.n_dir) {
    dl = f3(L.dir[l][0], L.dir[l][1], L.dir[l][2]);
    tmax = INFINITY;
  } else {
    int p = l - L.n_dir;
    float3 u = f3(L.pos[p][0], L.pos[p][1], L.pos[p][2]) - Xs;
    float dist = length(u);
    if (!(dist > 0.0f)) return false;
    dl = (1.0f / dist) * u;
    tmax = dist * (1.0f - 1e-6f);
  }
  return dot(ng, dl) > 0.0f;
}

// Nearest hit of every active probe ray, stored with the hit triangle's
// normal and material for the hit shading.  Front-face hits also queue their
// shadow rays: each wave counts its tasks, reserves one contiguous run of
// its task region with a single atomic add on the region's counter, and
// writes them light-major (the tasks of one light from one probe stay
// contiguous).  Where a wave's run lands depends on timing, what a task
// computes does not.  Every ray clears its visibility bytes.  The grid strides over
// the rays of all volumes (persistent when the grid is smaller than the ray
// count); the stride is a multiple of 64, so a wave always holds 64
// consecutive rays.
// The work index walks each probe's rays in the volume's coherent order
// (compact cones of the pattern, one per wave); results are stored by ray id.
__device__ __forceinline__ void trace_one(const VolumeSet& vs, const SceneGPU& sc, const LightSet& L,
                                          const FrameScratch& fs, const FrameCounters& C, int64_t work) {
  RaySlot s = locate_ray(vs, C, fs.active, work);
  const VolumeGPU& V = vs.v[s.v];
  const int r = V.order ? V.order[s.r] : s.r;
  const int64_t id = work - s.r + r;
  s.r = r;
  float3 o = slot_position(fs, s);
  float4 w = fs.omega[V.omega_base + s.r];
  float3 w3 = f3(w.x, w.y, w.z);
  Ray ray = make_ray(o, w3);
  float t;
  int tri = traverse<false, false>(sc, ray, INFINITY, t, dyn_stack + threadIdx.x, kTraceBlock);
  HitRec h;
  h.tri = tri;
  h.t = tri >= 0 ? t : INFINITY;
  h.mat = 0;
  h.pad = 0;
  float3 ng = f3(0.0f, 0.0f, 0.0f);
  if (tri >= 0) ng = tri_normal_material(sc, tri, h.mat);
  h.n[0] = ng.x;
  h.n[1] = ng.y;
  h.n[2] = ng.z;
  h.n[3] = 0.0f;
  fs.hits[id] = h;
  int nl = L.n_dir + L.n_point;
  if (nl == 0) return;
  bool front = false;
  float3 X;
  if (tri >= 0) {
    front = dot(w3, ng) <= 0.0f;
    X = f3(fmaf(h.t, w3.x, o.x), fmaf(h.t, w3.y, o.y), fmaf(h.t, w3.z, o.z));
  }
  const int lane = threadIdx.x & 63;
  uint32_t need_bits = 0;
  int n = 0;
  for (int l = 0; l < nl; l++) {
    fs.vis[(int64_t)l * fs.max_rays + id] = 0;
    bool need = false;
    if (front) {
      float3 Xs, dl;
      float tmax;
      need = shadow_ray(L, l, X, ng, Xs, dl, tmax);
    }
    need_bits |= (need ? 1u : 0u) << l;
    n += __popcll(__ballot(need));
  }
  if (n == 0) return;
  const int leader = __ffsll((long long)__ballot(1)) - 1;
  unsigned long long base = 0;
  const int64_t region = (work >> 6) & (kTaskRegions - 1);
  if (lane == leader)
    base = atomicAdd((unsigned long long*)&fs.counters->task_count[region], (unsigned long long)n);
  base = __shfl(base, leader);
  float4* run = fs.shadow_tasks + region * task_region_cap(fs.max_rays, nl) + (int64_t)base;
  int at = 0;
  for (int l = 0; l < nl; l++) {
    const bool need = (need_bits >> l) & 1u;
    const unsigned long long m = __ballot(need);
    if (need) {
      float3 Xs, dl;
      float tmax;
      shadow_ray(L, l, X, ng, Xs, dl, tmax);
      run[at + __popcll(m & ((1ull << lane) - 1ull))] =
          make_float4(Xs.x, Xs.y, Xs.z, __uint_as_float((uint32_t)(id << 5) | (uint32_t)l));
    }
    at += __popcll(m);
  }
}

__global__ __launch_bounds__(kTraceBlock) void k_trace(VolumeSet vs, SceneGPU sc, FrameScratch fs) {
  const FrameCounters& C = *fs.counters;
  const LightSet& L = fs.params->L;
  const int64_t total = C.ray_base[vs.n];
  for (int64_t work = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x; work < total;
       work += (int64_t)gridDim.x * kTraceBlock)
    trace_one(vs, sc, L, fs, C, work);
}

// The probe-ray trace of a frame with a batch of irradiance queries answered
// in the same launch, against the atlases and states the previous frame left
// (the trace reads no atlas and writes none, nor any probe state): blocks
// [0, trace_blocks) trace as k_trace does, striding over the rays; the rest
// take one query point per lane, in order.  The trace's waves wait on
// dependent node fetches, and the queries' arithmetic fills the issue slots
// they leave.
__global__ __launch_bounds__(kTraceBlock) void k_trace_query(VolumeSet vs, SceneGPU sc, FrameScratch fs,
                                                            int trace_blocks, QueryBatch q) {
  if ((int)blockIdx.x < trace_blocks) {
    const FrameCounters& C = *fs.counters;
    const LightSet& L = fs.params->L;
    const int64_t total = C.ray_base[vs.n];
    for (int64_t work = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x; work < total;
         work += (int64_t)trace_blocks * kTraceBlock)
      trace_one(vs, sc, L, fs, C, work);
  } else {
    const int64_t i = (int64_t)(blockIdx.x - trace_blocks) * kTraceBlock + threadIdx.x;
    if (i < q.n) query_point(vs, q.pos, q.nrm, q.view, q.first + i, q.out);
  }
}

// The shadow tasks in one dense order, region after region.  Lane r of the
// wave returns the number of tasks in the regions below r, `total` all of
// them.  Every lane of the wave must be active.
static_assert(kTaskRegions == 64, "one task region per lane");
__device__ __forceinline__ int64_t tasks_before_region(const FrameCounters& C, int64_t& total) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)C.task_count[lane];
  int64_t incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  total = __shfl(incl, 63);
  return incl - c;
}

// Index in the task array of task k of the dense order (k < total): the last
// region starting at or before k (an empty region starts where the next does
// and is passed over), by bisection over the lanes' `before`.  Every lane of
// the wave must be active.
__device__ __forceinline__ int64_t task_index(int64_t before, int64_t k, int64_t cap) {
  int r = 0;
#pragma unroll
  for (int step = kTaskRegions / 2; step > 0; step >>= 1)
    if (__shfl(before, r + step) <= k) r += step;
  return r * cap + (k - __shfl(before, r));
}

// Any-hit shadow rays over the dense task order.  Grid-stride over all
// tasks, a wave at a time (the index search needs every lane).
template <typename CNT>
__device__ __forceinline__ void shadow_one(const VolumeSet& vs, const SceneGPU& sc, const LightSet& L,
                                           const FrameScratch& fs, int64_t slot, CNT* cnt) {
  // the task carries the shadow origin computed at the hit, so the ray needs
  // no other load
  const float4 task = fs.shadow_tasks[slot];
  const uint32_t word = __float_as_uint(task.w);
  const int64_t id = word >> 5;
  const int l = word & 31;
  const float3 Xs = f3(task.x, task.y, task.z);
  Ray ray;
  float tmax;
  if (l < L.n_dir) {
    ray = make_ray(Xs, f3(L.dir[l][0], L.dir[l][1], L.dir[l][2]));
    tmax = INFINITY;
  } else {
    // A point light's segment is traced from the light toward the surface:
    // the same segment (to the shadow origin, whose float32 end lands within
    // a few ulps of it), and the rays of a wave -- one light, hit points of
    // neighbouring rays of one probe -- then share their origin and stay a
    // coherent bundle through the tree.
    const int p = l - L.n_dir;
    const float3 P = f3(L.pos[p][0], L.pos[p][1], L.pos[p][2]);
    const float3 u = P - Xs;
    const float dist = length(u);
    const float3 dl = (1.0f / dist) * u;
    tmax = dist;
    ray = make_ray(P, f3(-dl.x, -dl.y, -dl.z));
  }
  float t;
  int hit = traverse<true, false, CNT>(sc, ray, tmax, t, dyn_stack + threadIdx.x, kTraceBlock, cnt);
  if (!cnt && hit < 0) fs.vis[(int64_t)l * fs.max_rays + id] = 1;
}

// Any-hit shadow rays with lane refill.  Each wave owns one contiguous range
// of the dense task order, fixed by its index (no atomics); a lane whose ray
// has ended takes the range's next task at the next refill, so the wave's
// lanes stay busy until its range runs out, instead of waiting at every
// batch of 64 for the longest ray of the batch (after the persistent
// while-while traversal with replacement of terminated rays, Aila and Laine
// 2009).  A refill runs when at least `refill` lanes are idle (every lane
// of the wave takes part in it: the task index search reads other lanes).
// Each pass of the loop takes every active lane through its inner nodes to
// the next leaf (or the end), then that leaf's triangles.
// The ranges belong to the waves of the launch's first `shadow_blocks`
// workgroups (k_shadow_refill below).
__device__ __forceinline__ void refill_shadow_rays(const VolumeSet& vs, const SceneGPU& sc, const FrameScratch& fs,
                                                   int refill, int shadow_blocks) {
  const FrameCounters& C = *fs.counters;
  const LightSet& L = fs.params->L;
  int64_t total;
  const int64_t before = tasks_before_region(C, total);
  const int64_t cap = task_region_cap(fs.max_rays, L.n_dir + L.n_point);
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)shadow_blocks * (kTraceBlock / 64);
  const int64_t wave = (int64_t)blockIdx.x * (kTraceBlock / 64) + (threadIdx.x >> 6);
  const int64_t per = (total + waves - 1) / waves;
  int64_t next = wave * per;                  // the range's next task (same on every lane)
  const int64_t end = min(total, next + per);
  int* stack = dyn_stack + threadIdx.x;
  const int stride = kTraceBlock;
  bool active = false;
  Ray ray;
  float tmax = 0.0f;
  int node = 0, sp = 0;
  int64_t out = 0;                            // visibility byte of the lane's task
  while (true) {
    const unsigned long long idle = __ballot(!active);
    const int n_idle = __popcll(idle);
    if (next < end && (n_idle >= refill || n_idle == 64)) {
      const int rank = __popcll(idle & ((1ull << lane) - 1ull));
      const int64_t k = next + rank;
      const bool take = !active && k < end;
      const int64_t slot = task_index(before, take ? k : next, cap);
      if (take) {
        const float4 task = fs.shadow_tasks[slot];
        const uint32_t word = __float_as_uint(task.w);
        const int l = word & 31;
        const float3 Xs = f3(task.x, task.y, task.z);
        out = (int64_t)l * fs.max_rays + (int64_t)(word >> 5);
        if (l < L.n_dir) {
          ray = make_ray(Xs, f3(L.dir[l][0], L.dir[l][1], L.dir[l][2]));
          tmax = INFINITY;
        } else {
          // a point light's segment from the light (as in k_shadow)
          const int p = l - L.n_dir;
          const float3 P = f3(L.pos[p][0], L.pos[p][1], L.pos[p][2]);
          const float3 u = P - Xs;
          const float dist = length(u);
          const float3 dl = (1.0f / dist) * u;
          tmax = dist;
          ray = make_ray(P, f3(-dl.x, -dl.y, -dl.z));
        }
        node = sc.n_nodes > 0 ? 0 : kTraversalDone;
        sp = 0;
        active = true;
      }
      next += min((int64_t)n_idle, end - next);
    }
    if (__ballot(active) == 0) break;        // the range is used up (a refill of 64 idle lanes takes a task)
    if (!active) continue;
    // inner nodes to the next leaf (the step of traverse<>)
    while (node >= 0) {
      const float4* np = sc.nodes + (size_t)node * 4;
      float4 n0 = np[0], n1 = np[1], n2 = np[2], n3 = np[3];
      float t0, t1;
      const bool h0 = box_hit(ray, n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, tmax, t0);
      const bool h1 = box_hit(ray, n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, tmax, t1);
      const int l0 = bits_i(n3.x), l1 = bits_i(n3.y);
      const bool first0 = h0 & (!h1 | (t0 <= t1));
      const int nearc = first0 ? l0 : l1;
      const int farc = first0 ? l1 : l0;
      const int top = sp < sc.stack_depth - 1 ? sp : sc.stack_depth - 1;
      stack[top * stride] = farc;
      sp = top + ((h0 && h1) ? 1 : 0);
      const int below = sp > 0 ? sp - 1 : 0;
      const int popped = stack[below * stride];
      const bool any = h0 || h1;
      node = any ? nearc : (sp == 0 ? kTraversalDone : popped);
      sp = any ? sp : below;
    }
    bool done = node == kTraversalDone, hit = false;
    if (!done) {
      const int code = ~node;
      const int first = code >> 3, count = (code & 7) + 1;
      for (int i = first; i < first + count; i++) {
        const float4* tp = sc.tris + (size_t)i * 3;
        float t;
        if (tri_hit(ray, tp[0], tp[1], tp[2], tmax, t)) {
          hit = true;
          break;
        }
      }
      if (hit || sp == 0) {
        done = true;
      } else {
        sp--;
        node = stack[sp * stride];
      }
    }
    if (done) {
      if (!hit) fs.vis[out] = 1;
      active = false;
    }
  }
}

// A probe ray's front-face hit: the hit point, its normal and the ray
// direction (false for a miss or a backface).
__device__ __forceinline__ bool front_hit(const VolumeSet& vs, const FrameScratch& fs, const FrameCounters& C,
                                          int64_t id, const HitRec& h, float3& X, float3& ng, float3& w) {
  if (h.tri < 0) return false;
  const RaySlot s = locate_ray(vs, C, fs.active, id);
  const VolumeGPU& V = vs.v[s.v];
  const float3 o = slot_position(fs, s);
  const float4 w4 = fs.omega[V.omega_base + s.r];
  w = f3(w4.x, w4.y, w4.z);
  ng = f3(h.n[0], h.n[1], h.n[2]);
  if (dot(w, ng) > 0.0f) return false;
  X = f3(fmaf(h.t, w.x, o.x), fmaf(h.t, w.y, o.y), fmaf(h.t, w.z, o.z));
  return true;
}

// The indirect term of a front-face hit's shading: the previous frame's
// irradiance at the hit, queried from all volumes; it needs the hit alone,
// not the shadow rays, so it runs in the shadow-ray launch and waits in the
// ray's radiance slot for shade_one.
__device__ __forceinline__ void shade_indirect_one(const VolumeSet& vs, const FrameScratch& fs,
                                                   const FrameCounters& C, int64_t id) {
  const HitRec h = fs.hits[id];
  float3 X, ng, w;
  if (!front_hit(vs, fs, C, id, h, X, ng, w)) return;
  const float3 ind = query_irradiance(vs, X, ng, f3(-w.x, -w.y, -w.z));
  fs.rays[id] = make_float4(ind.x, ind.y, ind.z, 0.0f);
}

// Radiance and distance carried by each probe ray (backface rule of the
// self-shadow-bias section: radiance 0, distance shortened by 80 %).  IND:
// the indirect term of a front-face hit is already in the ray's radiance
// slot (shade_indirect_one ran); otherwise it is queried here.
template <bool IND>
__device__ __forceinline__ void shade_one(const VolumeSet& vs, const SceneGPU& sc, const LightSet& L,
                                          const FrameScratch& fs, const FrameCounters& C, int64_t id) {
  HitRec h = fs.hits[id];
  RaySlot s = locate_ray(vs, C, fs.active, id);
  const VolumeGPU& V = vs.v[s.v];
  float3 o = slot_position(fs, s);
  float4 w4 = fs.omega[V.omega_base + s.r];
  float3 w = f3(w4.x, w4.y, w4.z);
  // the visibility byte of every light, fetched up front and together (they
  // depend on the ray id alone): groups of eight unconditional loads (a light
  // index past the last reads the last light's byte again and is masked
  // off), one wait per group instead of one per light
  const int nl = L.n_dir + L.n_point;
  uint32_t vis = 0;
  for (int l0 = 0; l0 < nl; l0 += 8) {
    uint8_t b[8];
#pragma unroll
    for (int j = 0; j < 8; j++) b[j] = fs.vis[(int64_t)min(l0 + j, nl - 1) * fs.max_rays + id];
#pragma unroll
    for (int j = 0; j < 8; j++) vis |= (b[j] != 0 && l0 + j < nl ? 1u : 0u) << (l0 + j);
  }
  float4 out;
  if (h.tri < 0) {
    out = make_float4(L.sky[0], L.sky[1], L.sky[2], V.dmax);
  } else {
    const float3 ng = f3(h.n[0], h.n[1], h.n[2]);
    if (dot(w, ng) > 0.0f) {
      out = make_float4(0.0f, 0.0f, 0.0f, fminf(0.2f * h.t, V.dmax));
    } else {
      float3 X = f3(fmaf(h.t, w.x, o.x), fmaf(h.t, w.y, o.y), fmaf(h.t, w.z, o.z));
      float3 Xs = shadow_origin(X, ng);
      float3 direct = f3(0.0f, 0.0f, 0.0f);
      for (int l = 0; l < nl; l++) {
        if (!((vis >> l) & 1u)) continue;
        if (l < L.n_dir) {
          float c = dot(ng, f3(L.dir[l][0], L.dir[l][1], L.dir[l][2]));
          direct = direct + c * f3(L.irr[l][0], L.irr[l][1], L.irr[l][2]);
        } else {
          int p = l - L.n_dir;
          float3 u = f3(L.pos[p][0], L.pos[p][1], L.pos[p][2]) - Xs;
          float dist = length(u);
          float c = dot(ng, (1.0f / dist) * u);
          float k = c / (dist * dist);
          direct = direct + k * f3(L.irr[l][0], L.irr[l][1], L.irr[l][2]);
        }
      }
      float3 ind;
      if (IND) {
        const float4 r = fs.rays[id];
        ind = f3(r.x, r.y, r.z);
      } else {
        ind = query_irradiance(vs, X, ng, f3(-w.x, -w.y, -w.z));
      }
      float4 al = sc.albedo[h.mat], em = sc.emission[h.mat];
      const float inv_pi = 0.318309886183790672f;
      out = make_float4(fmaf(al.x, fmaf(direct.x, inv_pi, ind.x), em.x), fmaf(al.y, fmaf(direct.y, inv_pi, ind.y), em.y),
                        fmaf(al.z, fmaf(direct.z, inv_pi, ind.z), em.z), fminf(h.t, V.dmax));
    }
  }
  fs.rays[id] = out;
}

__global__ __launch_bounds__(kTraceBlock) void k_shade(VolumeSet vs, SceneGPU sc, FrameScratch fs) {
  const FrameCounters& C = *fs.counters;
  const LightSet& L = fs.params->L;
  const int64_t total = C.ray_base[vs.n];
  for (int64_t id = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x; id < total;
       id += (int64_t)gridDim.x * kTraceBlock)
    shade_one<false>(vs, sc, L, fs, C, id);
}

// The hit shading after the shadow-ray launch computed the indirect terms.
__global__ __launch_bounds__(kTraceBlock) void k_shade_direct(VolumeSet vs, SceneGPU sc, FrameScratch fs) {
  const FrameCounters& C = *fs.counters;
  const LightSet& L = fs.params->L;
  const int64_t total = C.ray_base[vs.n];
  for (int64_t id = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x; id < total;
       id += (int64_t)gridDim.x * kTraceBlock)
    shade_one<true>(vs, sc, L, fs, C, id);
}

// The shadow-ray launch (batched form): blocks [0, shadow_blocks) take the
// shadow tasks, 64 consecutive ones per wave, striding over the dense task
// order; the next hit_blocks stride over the probe rays and compute the
// indirect term of each front-face hit (shade_indirect_one: it reads the
// hit and the atlases, not the shadow rays); the rest, in k_shadow_query,
// take one point per lane of a share of a query batch against the atlases
// the previous frame left.  Nothing in this launch writes an atlas or a
// probe state.  The shadow rays' blocks come first, so they are resident
// from the start and the others fill the issue slots their traversal leaves.
__device__ __forceinline__ void shadow_stage(const VolumeSet& vs, const SceneGPU& sc, const FrameScratch& fs,
                                             int shadow_blocks, int hit_blocks, const QueryBatch& q) {
  const FrameCounters& C = *fs.counters;
  const int b = (int)blockIdx.x;
  if (b < shadow_blocks) {
    const LightSet& L = fs.params->L;
    int64_t total;
    const int64_t before = tasks_before_region(C, total);
    const int64_t cap = task_region_cap(fs.max_rays, L.n_dir + L.n_point);
    const int lane = threadIdx.x & 63;
    for (int64_t k0 = (int64_t)b * kTraceBlock + (threadIdx.x - lane); k0 < total;
         k0 += (int64_t)shadow_blocks * kTraceBlock) {
      const int64_t k = k0 + lane;
      const int64_t slot = task_index(before, k < total ? k : total - 1, cap);
      if (k < total) shadow_one<NoCount>(vs, sc, L, fs, slot, nullptr);
    }
  } else if (b < shadow_blocks + hit_blocks) {
    const int64_t total = C.ray_base[vs.n];
    for (int64_t id = (int64_t)(b - shadow_blocks) * kTraceBlock + threadIdx.x; id < total;
         id += (int64_t)hit_blocks * kTraceBlock)
      shade_indirect_one(vs, fs, C, id);
  } else {
    const int64_t i = (int64_t)(b - shadow_blocks - hit_blocks) * kTraceBlock + threadIdx.x;
    if (i < q.n) query_point(vs, q.pos, q.nrm, q.view, q.first + i, q.out);
  }
}

__global__ __launch_bounds__(kTraceBlock) void k_shadow(VolumeSet vs, SceneGPU sc, FrameScratch fs, int shadow_blocks,
                                                        int hit_blocks) {
  shadow_stage(vs, sc, fs, shadow_blocks, hit_blocks, QueryBatch{});
}

__global__ __launch_bounds__(kTraceBlock) void k_shadow_query(VolumeSet vs, SceneGPU sc, FrameScratch fs,
                                                             int shadow_blocks, int hit_blocks, QueryBatch q) {
  shadow_stage(vs, sc, fs, shadow_blocks, hit_blocks, q);
}

// The shadow rays with lane refill (refill_shadow_rays) on the first
// shadow_blocks workgroups and the hit shading's indirect terms on the next
// hit_blocks, as in shadow_stage.
__global__ __launch_bounds__(kTraceBlock) void k_shadow_refill(VolumeSet vs, SceneGPU sc, FrameScratch fs, int refill,
                                                               int shadow_blocks, int hit_blocks) {
  const int b = (int)blockIdx.x;
  if (b < shadow_blocks) {
    refill_shadow_rays(vs, sc, fs, refill, shadow_blocks);
  } else {
    const FrameCounters& C = *fs.counters;
    const int64_t total = C.ray_base[vs.n];
    for (int64_t id = (int64_t)(b - shadow_blocks) * kTraceBlock + threadIdx.x; id < total;
         id += (int64_t)hit_blocks * kTraceBlock)
      shade_indirect_one(vs, fs, C, id);
  }
}

// ---- classification (Section "Full Probe Initialization Algorithm")

struct ClassifyArgs {
  float R[IRF_MAX_ROTATIONS][9];
  int K;
  int64_t base[IRF_MAX_VOLUMES + 1];   // thread ranges per volume: P * K * N
};

// Whether probe q of volume v is selected by the mask (every probe when
// m.vol < 0; else the probes of volume m.vol on an entering plane).
__device__ __forceinline__ bool in_mask(const VolumeGPU& V, int v, int q, const PlaneMask& m) {
  if (m.vol < 0) return true;
  if (v != m.vol) return false;
  int g[3];
  logical_index(V, q, g);
  bool in = false;
  for (int a = 0; a < 3; a++) in = in || (g[a] >= m.lo[a] && g[a] <= m.hi[a]);
  return in;
}

__global__ __launch_bounds__(kTraceBlock) void k_classify(VolumeSet vs, SceneGPU sc, ClassifyArgs A, int32_t* back,
                                                          uint32_t* tfront, PlaneMask mask) {
  int64_t gid = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x;
  if (gid >= A.base[vs.n]) return;
  int v = 0;
  while (v + 1 < vs.n && gid >= A.base[v + 1]) v++;
  const VolumeGPU& V = vs.v[v];
  int64_t local = gid - A.base[v];
  int per_probe = A.K * V.rays;
  int q = (int)(local / per_probe);
  if (!in_mask(V, v, q, mask)) return;
  int rem = (int)(local - (int64_t)q * per_probe);
  int k = rem / V.rays, r = rem - k * V.rays;
  float3 o = probe_position(V, q);
  float3 w = sf_direction(r, V.rays, A.R[k]);
  Ray ray = make_ray(o, w);
  float t;
  int tri = traverse<false, true>(sc, ray, INFINITY, t, dyn_stack + threadIdx.x, kTraceBlock);
  if (tri < 0) return;
  int gq = V.probe_base + q;
  if (dot(w, tri_normal(sc, tri)) > 0.0f)
    atomicAdd(&back[gq], 1);
  else
    atomicMin(&tfront[gq], __float_as_uint(t));
}

__device__ __forceinline__ bool inside_grown_box(const VolumeGPU& V, ObjectBoxes ob, float3 P) {
  float D = fminf(V.spacing[0], fminf(V.spacing[1], V.spacing[2]));
  float b = 0.75f * D * V.bias;
  for (int o = 0; o < ob.n; o++) {
    bool in = true;
    float Pa[3] = {P.x, P.y, P.z};
    for (int a = 0; a < 3; a++) {
      float g = V.spacing[a] + b;
      in = in && Pa[a] >= ob.lo[3 * o + a] - g && Pa[a] <= ob.hi[3 * o + a] + g;
    }
    if (in) return true;
  }
  return false;
}

__global__ void k_classify_finish(VolumeSet vs, ObjectBoxes ob, int K, const int32_t* back, const uint32_t* tfront,
                                  PlaneMask mask) {
  int v = blockIdx.y;
  if (v >= vs.n) return;
  const VolumeGPU& V = vs.v[v];
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= V.n_probes) return;
  if (!in_mask(V, v, q, mask)) return;
  int gq = V.probe_base + q;
  float smax = fmaxf(V.spacing[0], fmaxf(V.spacing[1], V.spacing[2]));
  float tf = __uint_as_float(tfront[gq]);
  uint8_t st;
  if ((double)back[gq] / ((double)K * V.rays) > 0.25) st = IRF_OFF;
  else if (tf < smax) st = IRF_NEWLY_VIGILANT;
  else st = IRF_SLEEPING;
  if (st == IRF_SLEEPING && inside_grown_box(V, ob, probe_position(V, q))) st = IRF_NEWLY_AWAKE;
  V.states[q] = st;
}

// ---- second-order glossy (Section "Second Order Glossy")
//
// One thread per surface point: the mirror ray, its nearest hit, the hit's
// shadow rays, and the shading of the hit with the probes (irradiance at the
// hit; filtered radiance in the hit's own mirror direction for the further
// glossy bounces).

__global__ __launch_bounds__(kTraceBlock) void k_glossy(VolumeSet vs, SceneGPU sc, LightSet L,
                                                        const float* __restrict__ pos, const float* __restrict__ nrm,
                                                        const float* __restrict__ view, int64_t n,
                                                        float* __restrict__ out, irf_ray_record* rec) {
  const int64_t i = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x;
  if (i >= n) return;
  const float3 X = f3(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
  const float3 N = f3(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]);
  const float3 Vw = f3(view[3 * i], view[3 * i + 1], view[3 * i + 2]);
  const float c = dot(N, Vw);
  const float3 r = normalize_or_zero(f3(fmaf(2.0f * c, N.x, -Vw.x), fmaf(2.0f * c, N.y, -Vw.y),
                                        fmaf(2.0f * c, N.z, -Vw.z)));
  const float3 o = shadow_origin(X, N);
  float t;
  const int tri = traverse<false, false>(sc, make_ray(o, r), INFINITY, t, dyn_stack + threadIdx.x, kTraceBlock);
  float3 rgb = f3(0.0f, 0.0f, 0.0f);
  uint32_t vis = 0;
  if (tri < 0) {
    rgb = f3(L.sky[0], L.sky[1], L.sky[2]);
  } else {
    const float3 ng = tri_normal(sc, tri);
    if (dot(r, ng) <= 0.0f) {   // a backface is black
      const float3 Y = f3(fmaf(t, r.x, o.x), fmaf(t, r.y, o.y), fmaf(t, r.z, o.z));
      const float3 Ys = shadow_origin(Y, ng);
      float3 direct = f3(0.0f, 0.0f, 0.0f);
      const int nl = L.n_dir + L.n_point;
      for (int l = 0; l < nl; l++) {
        float3 Xs, dl;
        float tmax;
        if (!shadow_ray(L, l, Y, ng, Xs, dl, tmax)) continue;
        float ts;
        if (traverse<true, false>(sc, make_ray(Xs, dl), tmax, ts, dyn_stack + threadIdx.x, kTraceBlock) >= 0) continue;
        vis |= 1u << l;
        if (l < L.n_dir) {
          const float cl = dot(ng, f3(L.dir[l][0], L.dir[l][1], L.dir[l][2]));
          direct = direct + cl * f3(L.irr[l][0], L.irr[l][1], L.irr[l][2]);
        } else {
          const int p = l - L.n_dir;
          const float3 u = f3(L.pos[p][0], L.pos[p][1], L.pos[p][2]) - Ys;
          const float dist = length(u);
          const float cl = dot(ng, (1.0f / dist) * u);
          direct = direct + (cl / (dist * dist)) * f3(L.irr[l][0], L.irr[l][1], L.irr[l][2]);
        }
      }
      const float3 wo = f3(-r.x, -r.y, -r.z);
      const float3 E = query_irradiance(vs, Y, ng, wo);
      const float cr = dot(ng, r);
      const float3 r2 = f3(fmaf(-2.0f * cr, ng.x, r.x), fmaf(-2.0f * cr, ng.y, r.y), fmaf(-2.0f * cr, ng.z, r.z));
      const float3 G = query_look(vs, Y, ng, wo, r2);
      const int m = bits_i(sc.tris[(size_t)tri * 3 + 2].w);
      const float4 al = sc.albedo[m], em = sc.emission[m], sp = sc.specular[m];
      const float inv_pi = 0.318309886183790672f;
      rgb = f3(fmaf(sp.x, G.x, fmaf(al.x, fmaf(direct.x, inv_pi, E.x), em.x)),
               fmaf(sp.y, G.y, fmaf(al.y, fmaf(direct.y, inv_pi, E.y), em.y)),
               fmaf(sp.z, G.z, fmaf(al.z, fmaf(direct.z, inv_pi, E.z), em.z)));
    }
  }
  out[3 * i] = rgb.x;
  out[3 * i + 1] = rgb.y;
  out[3 * i + 2] = rgb.z;
  if (rec) {
    irf_ray_record q;
    q.tri = tri >= 0 ? bits_i(sc.tris[(size_t)tri * 3].w) : -1;
    q.t = tri >= 0 ? t : INFINITY;
    q.rgb[0] = rgb.x;
    q.rgb[1] = rgb.y;
    q.rgb[2] = rgb.z;
    q.d = 0.0f;
    q.vis = vis;
    q.probe = -1;
    rec[i] = q;
  }
}

void launch_glossy(const VolumeSet& vs, SceneGPU sc, const LightSet& L, const float* pos, const float* nrm,
                   const float* view, int64_t n, float* out, irf_ray_record* rec, hipStream_t s) {
  if (n == 0) return;
  irf_launch(k_glossy, dim3(blocks_for(n, kTraceBlock)), dim3(kTraceBlock), stack_bytes(sc), s, vs, sc, L, pos, nrm,
             view, n, out, rec);
}

// ---- tracking window: probes of entering planes start over (zero texels
// and offsets; the caller then classifies them)

__global__ void k_track_reset(VolumeSet vs, PlaneMask m) {
  const VolumeGPU& V = vs.v[m.vol];
  int q = blockIdx.x;
  if (q >= V.n_probes || !in_mask(V, m.vol, q, m)) return;
  const int es = V.atlas_f16 ? 2 : 4;
  uint32_t* irr = (uint32_t*)((char*)V.irr + (size_t)q * kIrrTexels * 4 * es);
  uint32_t* dist = (uint32_t*)((char*)V.dist + (size_t)q * kDistTexels * 2 * es);
  for (int i = threadIdx.x; i < kIrrTexels * es; i += blockDim.x) irr[i] = 0u;
  for (int i = threadIdx.x; i < kDistTexels * es / 2; i += blockDim.x) dist[i] = 0u;
  if (threadIdx.x < 3 && V.offsets) const_cast<float*>(V.offsets)[3 * q + threadIdx.x] = 0.0f;
}

void launch_track_reset(const VolumeSet& vs, PlaneMask m, hipStream_t s) {
  const int P = vs.v[m.vol].n_probes;
  if (P > 0) irf_launch(k_track_reset, dim3(P), dim3(256), 0, s, vs, m);
}

// ---- probe relocation (Section "Probe Position Adjustment")
//
// One iteration: every probe traces its rays (static geometry, one shared
// rotation) from its current position; per probe the backface count and
// three packed keys (t bits << 32 | ray) are reduced with atomics -- the
// closest backface and the closest front face (minimum), the farthest front
// face (maximum, ray stored complemented so ties keep the lowest ray) -- and
// k_reloc_finish moves the probe.

struct RelocArgs {
  float R[9];
  float limit;                          // offset limit, fraction of the spacing per axis
  int64_t base[IRF_MAX_VOLUMES + 1];    // ray ranges per volume: P * N
};

__global__ void k_reloc_init(int32_t* back, unsigned long long* keys, int64_t P) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < P; q += (int64_t)gridDim.x * blockDim.x) {
    back[q] = 0;
    keys[3 * q + 0] = ~0ull;
    keys[3 * q + 1] = ~0ull;
    keys[3 * q + 2] = 0ull;
  }
}

__global__ __launch_bounds__(kTraceBlock) void k_reloc_rays(VolumeSet vs, SceneGPU sc, RelocArgs A, int32_t* back,
                                                            unsigned long long* keys) {
  int64_t gid = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x;
  if (gid >= A.base[vs.n]) return;
  int v = 0;
  while (v + 1 < vs.n && gid >= A.base[v + 1]) v++;
  const VolumeGPU& V = vs.v[v];
  int64_t local = gid - A.base[v];
  int q = (int)(local / V.rays), r = (int)(local - (int64_t)q * V.rays);
  float3 w = sf_direction(r, V.rays, A.R);
  Ray ray = make_ray(probe_position(V, q), w);
  float t;
  int tri = traverse<false, true>(sc, ray, INFINITY, t, dyn_stack + threadIdx.x, kTraceBlock);
  if (tri < 0) return;
  const int64_t gq = V.probe_base + q;
  const unsigned long long tk = (unsigned long long)__float_as_uint(t) << 32;
  if (dot(w, tri_normal(sc, tri)) > 0.0f) {
    atomicAdd(&back[gq], 1);
    atomicMin(&keys[3 * gq + 0], tk | (unsigned)r);
  } else {
    atomicMin(&keys[3 * gq + 1], tk | (unsigned)r);
    atomicMax(&keys[3 * gq + 2], tk | (0xffffffffu - (unsigned)r));
  }
}

// Largest scale along v before an axis leaves [-lim, lim]; an axis with no
// component along v does not limit it.
__device__ __forceinline__ float axis_scale(float cur, float lim, float v) {
  if (v == 0.0f) return INFINITY;
  return fmaxf((lim - cur) / v, (-lim - cur) / v);
}

__global__ void k_reloc_finish(VolumeSet vs, RelocArgs A, const int32_t* back, const unsigned long long* keys) {
  int v = blockIdx.y;
  if (v >= vs.n) return;
  const VolumeGPU& V = vs.v[v];
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= V.n_probes) return;
  const int64_t gq = V.probe_base + q;
  float* off = const_cast<float*>(V.offsets) + 3 * q;
  const float cur[3] = {off[0], off[1], off[2]};
  float lim[3];
  for (int a = 0; a < 3; a++) lim[a] = A.limit * V.spacing[a];
  const int N = V.rays;
  float nw[3] = {cur[0], cur[1], cur[2]};
  if (4 * back[gq] > N) {
    // more than 25 % backfaces: through the closest backface, as far as the
    // offset limit allows (less 1e-3 of the scale), only if that gets through
    const unsigned long long k = keys[3 * gq + 0];
    const float t = __uint_as_float((unsigned)(k >> 32));
    const float3 w = sf_direction((int)(k & 0xffffffffu), N, A.R);
    const float vv[3] = {t * w.x, t * w.y, t * w.z};
    float sc = INFINITY;
    for (int a = 0; a < 3; a++) sc = fminf(sc, axis_scale(cur[a], lim[a], vv[a]));
    sc -= 1e-3f;
    if (sc > 1.0f)
      for (int a = 0; a < 3; a++) nw[a] = cur[a] + vv[a] * sc;
  } else if (keys[3 * gq + 2] != 0ull) {
    // a bounded step toward the farthest front face, unless it lies within
    // 60 degrees of the closest one (the probe sees one surface)
    const unsigned long long kf = keys[3 * gq + 2], kc = keys[3 * gq + 1];
    const float tf = __uint_as_float((unsigned)(kf >> 32));
    const float3 wf = sf_direction((int)(0xffffffffu - (unsigned)(kf & 0xffffffffu)), N, A.R);
    const float3 wc = sf_direction((int)(kc & 0xffffffffu), N, A.R);
    if (!(dot(wf, wc) > 0.5f)) {
      const float step = fminf(0.2f, tf);
      const float cand[3] = {cur[0] + step * wf.x, cur[1] + step * wf.y, cur[2] + step * wf.z};
      bool inside = true;
      for (int a = 0; a < 3; a++) inside = inside && fabsf(cand[a]) <= lim[a];
      if (inside)
        for (int a = 0; a < 3; a++) nw[a] = cand[a];
    }
  }
  off[0] = nw[0];
  off[1] = nw[1];
  off[2] = nw[2];
}

void launch_relocate(const VolumeSet& vs, SceneGPU sc, const float* rotation, float limit, int32_t* back,
                     unsigned long long* keys, hipStream_t s) {
  RelocArgs A;
  for (int i = 0; i < 9; i++) A.R[i] = rotation[i];
  A.limit = limit;
  A.base[0] = 0;
  int64_t P = 0;
  int maxp = 0;
  for (int v = 0; v < vs.n; v++) {
    A.base[v + 1] = A.base[v] + (int64_t)vs.v[v].n_probes * vs.v[v].rays;
    P += vs.v[v].n_probes;
    maxp = vs.v[v].n_probes > maxp ? vs.v[v].n_probes : maxp;
  }
  if (P == 0) return;
  irf_launch(k_reloc_init, dim3(blocks_for(P, 256)), dim3(256), 0, s, back, keys, P);
  irf_launch(k_reloc_rays, dim3(blocks_for(A.base[vs.n], kTraceBlock)), dim3(kTraceBlock), stack_bytes(sc), s, vs,
             sc, A, back, keys);
  irf_launch(k_reloc_finish, dim3(blocks_for(maxp, 256), vs.n), dim3(256), 0, s, vs, A, (const int32_t*)back,
             (const unsigned long long*)keys);
}

// ---- traversal statistics (on demand): node and triangle fetches of the
// last frame's probe rays (out[0..1]) and shadow rays (out[2..3])

__device__ __forceinline__ void add_block(unsigned long long* out, unsigned long long v) {
  // one atomic per wave
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(out, v);
}

__global__ __launch_bounds__(kTraceBlock) void k_trace_count(VolumeSet vs, SceneGPU sc, FrameScratch fs,
                                                             unsigned long long* out) {
  const FrameCounters& C = *fs.counters;
  int64_t id = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x;
  Count cnt;
  if (id < C.ray_base[vs.n]) {
    RaySlot s = locate_ray(vs, C, fs.active, id);
    const VolumeGPU& V = vs.v[s.v];
    float4 w = fs.omega[V.omega_base + s.r];
    Ray ray = make_ray(slot_position(fs, s), f3(w.x, w.y, w.z));
    float t;
    traverse<false, false, Count>(sc, ray, INFINITY, t, dyn_stack + threadIdx.x, kTraceBlock, &cnt);
  }
  add_block(&out[0], cnt.nodes);
  add_block(&out[1], cnt.tris);
}

__global__ __launch_bounds__(kTraceBlock) void k_shadow_count(VolumeSet vs, SceneGPU sc, FrameScratch fs,
                                                              unsigned long long* out) {
  const FrameCounters& C = *fs.counters;
  const LightSet& L = fs.params->L;
  int64_t total;
  const int64_t before = tasks_before_region(C, total);
  const int64_t k = (int64_t)blockIdx.x * kTraceBlock + threadIdx.x;
  Count cnt;
  if (total > 0) {
    const int64_t slot = task_index(before, k < total ? k : total - 1, task_region_cap(fs.max_rays, L.n_dir + L.n_point));
    if (k < total) shadow_one<Count>(vs, sc, L, fs, slot, &cnt);
  }
  add_block(&out[2], cnt.nodes);
  add_block(&out[3], cnt.tris);
}

void launch_traversal_stats(const VolumeSet& vs, SceneGPU sc, int n_lights, FrameScratch fs, unsigned long long* out,
                            hipStream_t s) {
  irf_launch(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)out, 0u, (int64_t)8);
  if (fs.max_rays == 0) return;
  irf_launch(k_trace_count, dim3(blocks_for(fs.max_rays, kTraceBlock)), dim3(kTraceBlock), stack_bytes(sc), s,
                     vs, sc, fs, out);
  if (n_lights == 0) return;
  int64_t cap = (fs.max_rays + 63) / 64 * 64 * n_lights;
  irf_launch(k_shadow_count, dim3(blocks_for(cap, kTraceBlock)), dim3(kTraceBlock), stack_bytes(sc), s, vs, sc,
                     fs, out);
}

// ---- frame statistics (on demand, outside the frame)

__global__ void k_frame_stats(VolumeSet vs, SceneGPU sc, FrameScratch fs, unsigned long long* out) {
  const FrameCounters& C = *fs.counters;
  int64_t total = C.ray_base[vs.n];
  unsigned long long tasks = 0, front = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    HitRec h = fs.hits[i];
    if (h.tri >= 0) {
      RaySlot s = locate_ray(vs, C, fs.active, i);
      float4 w = fs.omega[vs.v[s.v].omega_base + s.r];
      if (dot(f3(w.x, w.y, w.z), tri_normal(sc, h.tri)) <= 0.0f) front++;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int r = 0; r < kTaskRegions; r++) tasks += (unsigned long long)C.task_count[r];
  atomicAdd(&out[0], tasks);
  atomicAdd(&out[1], front);
}

void launch_frame_stats(const VolumeSet& vs, SceneGPU sc, FrameScratch fs, unsigned long long* out, hipStream_t s) {
  irf_launch(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)out, 0u, (int64_t)4);
  irf_launch(k_frame_stats, dim3(256), dim3(256), 0, s, vs, sc, fs, out);
}

// ---- debug records

__global__ void k_records(VolumeSet vs, int vol, SceneGPU sc, FrameScratch fs, int n_lights, irf_ray_record* out,
                          int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const FrameCounters& C = *fs.counters;
  int64_t id = C.ray_base[vol] + i;
  const VolumeGPU& V = vs.v[vol];
  HitRec h = fs.hits[id];
  float4 r = fs.rays[id];
  irf_ray_record rec;
  rec.tri = h.tri >= 0 ? bits_i(sc.tris[(size_t)h.tri * 3].w) : -1;
  rec.t = h.t;
  rec.rgb[0] = r.x;
  rec.rgb[1] = r.y;
  rec.rgb[2] = r.z;
  rec.d = r.w;
  uint32_t vis = 0;
  for (int l = 0; l < n_lights; l++)
    if (fs.vis[(int64_t)l * fs.max_rays + id]) vis |= 1u << l;
  rec.vis = vis;
  rec.probe = fs.active[C.slot_base[vol] + (int)(i / V.rays)] - V.probe_base;
  out[i] = rec;
}

// ---- launches

// grid: 0 = one block per 128 items of the largest possible frame;
// otherwise a persistent grid of that many blocks striding over the items
static inline unsigned grid_for(int64_t items, int grid) {
  unsigned full = blocks_for(items, kTraceBlock);
  if (grid <= 0 || (unsigned)grid > full) return full > 0 ? full : 1;
  return (unsigned)grid;
}

void launch_trace(const VolumeSet& vs, SceneGPU sc, FrameScratch fs, int grid, hipStream_t s) {
  if (fs.max_rays == 0) return;
  irf_launch(k_trace, dim3(grid_for(fs.max_rays, grid)), dim3(kTraceBlock), stack_bytes(sc), s, vs, sc, fs);
}

void launch_trace_query(const VolumeSet& vs, SceneGPU sc, FrameScratch fs, int grid, const QueryBatch& q,
                        hipStream_t s) {
  if (q.n == 0) return launch_trace(vs, sc, fs, grid, s);
  const unsigned tb = fs.max_rays > 0 ? grid_for(fs.max_rays, grid) : 0;
  const unsigned qb = blocks_for(q.n, kTraceBlock);
  irf_launch(k_trace_query, dim3(tb + qb), dim3(kTraceBlock), stack_bytes(sc), s, vs, sc, fs, (int)tb, q);
}

void launch_shadow(const VolumeSet& vs, SceneGPU sc, int n_lights, FrameScratch fs, int grid, int hit_grid,
                   int refill, hipStream_t s) {
  if (fs.max_rays == 0 || n_lights == 0) return;
  const int64_t cap = (fs.max_rays + 63) / 64 * 64 * n_lights;
  const unsigned sb = grid_for(cap, grid), hb = grid_for(fs.max_rays, hit_grid);
  irf_launch(k_shadow_refill, dim3(sb + hb), dim3(kTraceBlock), stack_bytes(sc), s, vs, sc, fs,
             refill > 0 ? refill : 64, (int)sb, (int)hb);
}

void launch_shadow_stage(const VolumeSet& vs, SceneGPU sc, int n_lights, FrameScratch fs, int grid, int hit_grid,
                         const QueryBatch& q, hipStream_t s) {
  const int64_t cap = (fs.max_rays + 63) / 64 * 64 * n_lights;
  const unsigned sb = fs.max_rays > 0 && n_lights > 0 ? grid_for(cap, grid) : 0;
  const unsigned hb = fs.max_rays > 0 ? grid_for(fs.max_rays, hit_grid) : 0;
  const unsigned qb = blocks_for(q.n, kTraceBlock);
  if (sb + hb + qb == 0) return;
  if (q.n > 0)
    irf_launch(k_shadow_query, dim3(sb + hb + qb), dim3(kTraceBlock), stack_bytes(sc), s, vs, sc, fs, (int)sb,
               (int)hb, q);
  else
    irf_launch(k_shadow, dim3(sb + hb), dim3(kTraceBlock), stack_bytes(sc), s, vs, sc, fs, (int)sb, (int)hb);
}

void launch_shade(const VolumeSet& vs, SceneGPU sc, FrameScratch fs, int grid, bool indirect_done, hipStream_t s) {
  if (fs.max_rays == 0) return;
  if (indirect_done)
    irf_launch(k_shade_direct, dim3(grid_for(fs.max_rays, grid)), dim3(kTraceBlock), 0, s, vs, sc, fs);
  else
    irf_launch(k_shade, dim3(grid_for(fs.max_rays, grid)), dim3(kTraceBlock), 0, s, vs, sc, fs);
}

void launch_classify(const VolumeSet& vs, SceneGPU sc, ObjectBoxes boxes, const float* rotations, int K,
                     int32_t* back, uint32_t* tfront, PlaneMask mask, hipStream_t s) {
  ClassifyArgs A;
  for (int k = 0; k < K; k++)
    for (int i = 0; i < 9; i++) A.R[k][i] = rotations[9 * k + i];
  A.K = K;
  A.base[0] = 0;
  int total_probes = 0;
  for (int v = 0; v < vs.n; v++) {
    A.base[v + 1] = A.base[v] + (int64_t)vs.v[v].n_probes * K * vs.v[v].rays;
    total_probes += vs.v[v].n_probes;
  }
  irf_launch(k_fill_u32, dim3(blocks_for(total_probes, 256)), dim3(256), 0, s, (uint32_t*)back, 0u,
                     (int64_t)total_probes);
  irf_launch(k_fill_u32, dim3(blocks_for(total_probes, 256)), dim3(256), 0, s, tfront,
                     (uint32_t)0x7f800000u, (int64_t)total_probes);
  if (A.base[vs.n] > 0)
    irf_launch(k_classify, dim3(blocks_for(A.base[vs.n], kTraceBlock)), dim3(kTraceBlock), stack_bytes(sc), s,
                       vs, sc, A, back, tfront, mask);
  int maxp = 0;
  for (int v = 0; v < vs.n; v++) maxp = vs.v[v].n_probes > maxp ? vs.v[v].n_probes : maxp;
  irf_launch(k_classify_finish, dim3(blocks_for(maxp, 256), vs.n), dim3(256), 0, s, vs, boxes, K, back,
                     tfront, mask);
}

void launch_records(const VolumeSet& vs, int vol, SceneGPU sc, FrameScratch fs, int n_lights, irf_ray_record* out,
                    int64_t count, hipStream_t s) {
  if (count == 0) return;
  irf_launch(k_records, dim3(blocks_for(count, 256)), dim3(256), 0, s, vs, vol, sc, fs, n_lights, out, count);
}

}  // namespace irf
