// C ABI of the irf library: argument validation, ownership of the scene and
// frame scratch, and the launch sequence of one update frame.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "irf_internal.h"

namespace irf {
thread_local KernelTiming* g_kernel_timing = nullptr;
}

using namespace irf;

namespace {

thread_local std::string g_err;

irf_status fail(irf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(IRF_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool finite3(const float* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  irf_status reserve(size_t count) {
    if (count <= n && p) return IRF_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    if (count == 0) return IRF_OK;
    hipError_t e = hipMalloc((void**)&p, sizeof(T) * count);
    if (e != hipSuccess) {
      p = nullptr;
      return fail(IRF_E_NOMEM, "hipMalloc(%zu bytes) failed: %s", sizeof(T) * count, hipGetErrorString(e));
    }
    n = count;
    return IRF_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

}  // namespace

struct irf_ctx {
  int device = 0;
  // scene
  bool has_scene = false;
  DevBuf<float4> nodes, tris, albedo, emission, specular;
  DevBuf<float> obj_lo, obj_hi;
  int32_t n_tris = 0, n_nodes = 0, n_materials = 0, n_obj = 0;
  double bvh_stats[5] = {0, 0, 0, 0, 0};
  // lights
  LightSet lights;
  // volumes
  int32_t n_vol = 0;
  irf_volume_desc desc[IRF_MAX_VOLUMES];
  VolumeGPU vol[IRF_MAX_VOLUMES];
  bool bound[IRF_MAX_VOLUMES];
  // frame scratch
  DevBuf<FrameParams> params;
  DevBuf<int32_t> block_active;
  DevBuf<int32_t> active;
  DevBuf<FrameCounters> counters;
  DevBuf<float4> omega;
  DevBuf<int16_t> order;           // per volume at omega_base: coherent trace order of its rays
  std::vector<int32_t> order_rays;  // ray counts the order was built for
  DevBuf<HitRec> hits;
  DevBuf<uint8_t> vis;
  DevBuf<float4> rays;
  DevBuf<float4> shadow_tasks;
  DevBuf<unsigned long long> stats;
  DevBuf<char> weights;
  DevBuf<float> inv_row_sum;
  DevBuf<int32_t> class_back;
  DevBuf<uint32_t> class_tf;
  DevBuf<unsigned long long> reloc_keys;
  bool frame_done = false;
  bool diff_frame = false;   // the last frame saved its inputs for the adjoint
  Tuning tune = {0, 0, 0, 0, 0, 0, 500};
  // adjoint: the frame's input atlases and states, saved by each update
  bool diff = false;
  DevBuf<char> saved;
  int64_t saved_irr[IRF_MAX_VOLUMES], saved_dist[IRF_MAX_VOLUMES], saved_states[IRF_MAX_VOLUMES];
  DevBuf<float4> grad_rays;
  DevBuf<float4> probe_pos;
  DevBuf<char> adj;        // the adjoint's term buffers, segments and sort storage
  // kernel timing
  bool prof = false;
  struct ProfRec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  std::map<std::string, std::pair<int64_t, double>> prof_acc;
};

namespace {

irf_status set_device(const irf_ctx* c) {
  HIP_TRY(hipSetDevice(c->device));
  return IRF_OK;
}

SceneGPU scene_view(const irf_ctx* c) {
  SceneGPU s;
  memset(&s, 0, sizeof(s));   // padding too: frame_signature hashes the bytes
  s.nodes = c->nodes.p;
  s.tris = c->tris.p;
  s.albedo = c->albedo.p;
  s.emission = c->emission.p;
  s.specular = c->specular.p;
  s.n_tris = c->n_tris;
  s.n_nodes = c->n_nodes;
  s.stack_depth = (int32_t)c->bvh_stats[2];
  return s;
}

ObjectBoxes boxes_view(const irf_ctx* c) {
  ObjectBoxes b;
  memset(&b, 0, sizeof(b));
  b.lo = c->obj_lo.p;
  b.hi = c->obj_hi.p;
  b.n = c->n_obj;
  return b;
}

VolumeSet volume_view(const irf_ctx* c) {
  VolumeSet vs;
  memset(&vs, 0, sizeof(vs));
  vs.n = c->n_vol;
  const bool ordered = (int)c->order_rays.size() == c->n_vol && c->order.p;
  for (int v = 0; v < c->n_vol; v++) {
    vs.v[v] = c->vol[v];
    vs.v[v].order = ordered ? c->order.p + c->vol[v].omega_base : nullptr;
  }
  return vs;
}

// Order in which the probe-ray traversal takes the N rays of a probe: the
// unrotated spherical-Fibonacci directions grouped into N / 64 compact cones
// (greedy balanced assignment, nearest first, to the directions of an
// (N / 64)-point pattern), so that a wave traces one cone rather than a band
// of the sphere; the frame's rotation keeps the cones compact.  Only the lane
// a ray runs on changes: every ray keeps its index and result.
void coherent_order(int N, int16_t* out) {
  const int G = N / 64;
  if (G <= 1) {
    for (int i = 0; i < N; i++) out[i] = (int16_t)i;
    return;
  }
  auto dir = [](int i, int n, double w[3]) {
    const double z = 1.0 - (2.0 * i + 1.0) / n, r = std::sqrt(std::max(0.0, 1.0 - z * z));
    const double f = std::fmod(i * 0.61803398874989484820, 1.0), phi = 6.28318530717958647692 * f;
    w[0] = r * std::cos(phi);
    w[1] = r * std::sin(phi);
    w[2] = z;
  };
  std::vector<double> d(3 * (size_t)N), cen(3 * (size_t)G);
  for (int i = 0; i < N; i++) dir(i, N, &d[3 * i]);
  for (int g = 0; g < G; g++) dir(g, G, &cen[3 * g]);
  struct Pair {
    double c;
    int i, g;
  };
  std::vector<Pair> pairs;
  pairs.reserve((size_t)N * G);
  for (int i = 0; i < N; i++)
    for (int g = 0; g < G; g++)
      pairs.push_back({d[3 * i] * cen[3 * g] + d[3 * i + 1] * cen[3 * g + 1] + d[3 * i + 2] * cen[3 * g + 2], i, g});
  std::stable_sort(pairs.begin(), pairs.end(), [](const Pair& a, const Pair& b) { return a.c > b.c; });
  const int cap = (N + G - 1) / G;
  std::vector<int> group(N, -1), count(G, 0);
  for (const Pair& p : pairs)
    if (group[p.i] < 0 && count[p.g] < cap) {
      group[p.i] = p.g;
      count[p.g]++;
    }
  int k = 0;
  for (int g = 0; g < G; g++)
    for (int i = 0; i < N; i++)
      if (group[i] == g) out[k++] = (int16_t)i;
}

int64_t total_probes(const irf_ctx* c) {
  int64_t p = 0;
  for (int v = 0; v < c->n_vol; v++) p += c->vol[v].n_probes;
  return p;
}

int64_t total_rays(const irf_ctx* c) {
  int64_t r = 0;
  for (int v = 0; v < c->n_vol; v++) r += (int64_t)c->vol[v].n_probes * c->vol[v].rays;
  return r;
}

irf_status ensure_scratch(irf_ctx* c) {
  irf_status s;
  int64_t P = total_probes(c), R = total_rays(c);
  int nl = c->lights.n_dir + c->lights.n_point;
  if (R >= (1ll << 27)) return fail(IRF_E_UNSUPPORTED, "too many rays per frame (%lld >= 2^27)", (long long)R);
  int64_t om = 0;
  for (int v = 0; v < c->n_vol; v++) om += c->vol[v].rays;
  if ((s = c->params.reserve(1)) != IRF_OK) return s;
  if ((s = c->active.reserve((size_t)P)) != IRF_OK) return s;
  if ((s = c->probe_pos.reserve((size_t)(P > 0 ? P : 1))) != IRF_OK) return s;
  int64_t nb = 0;
  for (int v = 0; v < c->n_vol; v++) nb += (c->vol[v].n_probes + 1023) / 1024;
  if ((s = c->block_active.reserve((size_t)(nb > 0 ? nb : 1))) != IRF_OK) return s;
  if ((s = c->counters.reserve(1)) != IRF_OK) return s;
  if ((s = c->omega.reserve((size_t)om)) != IRF_OK) return s;
  std::vector<int32_t> rays_now(c->n_vol);
  for (int v = 0; v < c->n_vol; v++) rays_now[v] = c->vol[v].rays;
  if (rays_now != c->order_rays) {
    std::vector<int16_t> h((size_t)(om > 0 ? om : 1));
    for (int v = 0; v < c->n_vol; v++) coherent_order(c->vol[v].rays, &h[c->vol[v].omega_base]);
    c->order_rays.clear();
    if ((s = c->order.reserve(h.size())) != IRF_OK) return s;
    HIP_TRY(hipMemcpy(c->order.p, h.data(), h.size() * sizeof(int16_t), hipMemcpyHostToDevice));
    c->order_rays = rays_now;
  }
  if ((s = c->hits.reserve((size_t)R)) != IRF_OK) return s;
  if ((s = c->vis.reserve((size_t)R * (size_t)(nl > 0 ? nl : 1))) != IRF_OK) return s;
  if ((s = c->rays.reserve((size_t)R)) != IRF_OK) return s;
  if ((s = c->shadow_tasks.reserve((size_t)(kTaskRegions * task_region_cap(R, nl > 0 ? nl : 1)))) != IRF_OK)
    return s;
  if ((s = c->stats.reserve(8)) != IRF_OK) return s;
  if (c->diff) {
    int64_t off = 0;
    for (int v = 0; v < c->n_vol; v++) {
      int64_t P = c->vol[v].n_probes, es = c->vol[v].atlas_f16 ? 2 : 4;
      c->saved_irr[v] = off;
      off += (P * kIrrTexels * 4 * es + 255) / 256 * 256;
      c->saved_dist[v] = off;
      off += (P * kDistTexels * 2 * es + 255) / 256 * 256;
      c->saved_states[v] = off;
      off += (P + 255) / 256 * 256;
    }
    if ((s = c->saved.reserve((size_t)off)) != IRF_OK) return s;
    if ((s = c->grad_rays.reserve((size_t)(R > 0 ? R : 1))) != IRF_OK) return s;
  }
  int64_t wbytes = 0;
  for (int v = 0; v < c->n_vol; v++) wbytes += 256ll * c->vol[v].rays * 4;
  if ((s = c->weights.reserve((size_t)(wbytes > 0 ? wbytes : 16))) != IRF_OK) return s;
  if ((s = c->inv_row_sum.reserve((size_t)256 * (c->n_vol > 0 ? c->n_vol : 1))) != IRF_OK) return s;
  return IRF_OK;
}

FrameScratch scratch_view(const irf_ctx* c) {
  FrameScratch f;
  memset(&f, 0, sizeof(f));   // padding too: frame_signature hashes the bytes
  f.params = c->params.p;
  f.block_active = c->block_active.p;
  f.active = c->active.p;
  f.counters = c->counters.p;
  f.omega = c->omega.p;
  f.hits = c->hits.p;
  f.vis = c->vis.p;
  f.rays = c->rays.p;
  f.shadow_tasks = c->shadow_tasks.p;
  f.grad_rays = c->grad_rays.p;
  f.probe_pos = c->probe_pos.p;
  f.weights = c->weights.p;
  f.inv_row_sum = c->inv_row_sum.p;
  f.max_rays = total_rays(c);
  f.max_slots = (int32_t)total_probes(c);
  return f;
}

irf_status check_ready(const irf_ctx* c) {
  if (!c->has_scene) return fail(IRF_E_STATE, "no scene: call irf_set_scene first");
  if (c->n_vol == 0) return fail(IRF_E_STATE, "no volume: call irf_create_volume first");
  for (int v = 0; v < c->n_vol; v++)
    if (!c->bound[v]) return fail(IRF_E_STATE, "volume %d has no bound buffers (irf_bind_volume)", v);
  return IRF_OK;
}

hipEvent_t prof_event(irf_ctx* c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// While timing is enabled, times the kernels launched in its scope with
// events stamped on their dispatches.
struct ProfScope {
  irf_ctx* c;
  const char* name;
  KernelTiming t;
  KernelTiming* outer;
  bool on = false;
  ProfScope(irf_ctx* c_, const char* n, hipStream_t) : c(c_), name(n), outer(g_kernel_timing) {
    if (!c->prof) return;
    t.start = prof_event(c);
    t.stop = prof_event(c);
    t.first = true;
    if (t.start && t.stop) {
      on = true;
      g_kernel_timing = &t;
    } else {
      if (t.start) c->prof_pool.push_back(t.start);
      if (t.stop) c->prof_pool.push_back(t.stop);
    }
  }
  ~ProfScope() {
    if (!on) return;
    g_kernel_timing = outer;
    if (!t.first) {
      c->prof_pending.push_back({name, t.start, t.stop});
    } else {   // nothing was launched
      c->prof_pool.push_back(t.start);
      c->prof_pool.push_back(t.stop);
    }
  }
};

irf_status launched() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(IRF_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return IRF_OK;
}

// One update frame, asynchronously on `st` (also what a graph captures); the
// blend waits for `atlas_wait` when given.  With a query batch `qb` the
// queries see the atlases and states as they stood before the frame: they run
// inside the probe-ray trace and shadow-ray launches, or first, on their own,
// when the state step can rewrite the states they read.
hipError_t enqueue_frame_on(irf_ctx* c, const float* rotation, hipStream_t st, hipEvent_t atlas_wait,
                            const VolumeSet& vs, const FrameScratch& fs, const QueryBatch* qb = nullptr) {
  SceneGPU sc = scene_view(c);
  const int nl = c->lights.n_dir + c->lights.n_point;
  FrameParams fp;
  for (int i = 0; i < 9; i++) fp.R[i] = rotation[i];
  fp.L = c->lights;
  bool any_mma = false, any_valu = false;
  for (int v = 0; v < c->n_vol; v++) (c->vol[v].blend == IRF_BLEND_F32_VALU ? any_valu : any_mma) = true;
  // With dynamic objects in the scene the state step rewrites probe states
  // (an Awake probe away from every object goes to sleep), which the queries
  // read: then the whole frame waits, not only its atlas writes.
  const ObjectBoxes boxes = boxes_view(c);
  if (atlas_wait && boxes.n > 0) {
    hipError_t e = hipStreamWaitEvent(st, atlas_wait, 0);
    if (e != hipSuccess) return e;
    atlas_wait = nullptr;
  }
  const bool fused = qb && qb->n > 0 && boxes.n == 0;
  if (qb && qb->n > 0 && !fused) {
    ProfScope p(c, "query", st);
    launch_query(vs, qb->pos, qb->nrm, qb->view, qb->n, qb->out, st);
  }
  {
    ProfScope p(c, "frame_begin", st);
    launch_frame_begin(make_frame_begin(fp, vs, boxes, fs, any_mma), st);
  }
  if (c->diff) {
    // the frame's inputs for the adjoint: atlases and the stepped states
    for (int v = 0; v < c->n_vol; v++) {
      int64_t P = c->vol[v].n_probes, es = c->vol[v].atlas_f16 ? 2 : 4;
      launch_copy(c->saved.p + c->saved_irr[v], c->vol[v].irr, P * kIrrTexels * 4 * es, st);
      launch_copy(c->saved.p + c->saved_dist[v], c->vol[v].dist, P * kDistTexels * 2 * es, st);
      launch_copy(c->saved.p + c->saved_states[v], c->vol[v].states, P, st);
    }
  }
  // The shadow rays share their launch with the hit shading's indirect terms
  // and, in batches (`stage`), with the tuning's share of a fused query batch;
  // the rest of the batch runs in the trace launch.  With no light the hit
  // shading queries the indirect terms itself.
  const bool stage = nl > 0 && c->tune.shadow_refill == 0;
  QueryBatch q_shadow = {};
  if (fused) {
    const int64_t ns = stage ? qb->n * c->tune.query_shadow / 1000 : 0;
    QueryBatch q_trace = *qb;
    q_trace.n = qb->n - ns;
    q_shadow = *qb;
    q_shadow.first = qb->first + q_trace.n;
    q_shadow.n = ns;
    ProfScope p(c, "trace_query", st);
    launch_trace_query(vs, sc, fs, c->tune.trace_blocks, q_trace, st);
  } else {
    ProfScope p(c, "trace", st);
    launch_trace(vs, sc, fs, c->tune.trace_blocks, st);
  }
  if (stage) {
    ProfScope p(c, q_shadow.n > 0 ? "shadow_query" : "shadow", st);
    launch_shadow_stage(vs, sc, nl, fs, c->tune.shadow_blocks, c->tune.shade_blocks, q_shadow, st);
  } else if (nl > 0) {
    ProfScope p(c, "shadow_refill", st);
    launch_shadow(vs, sc, nl, fs, c->tune.shadow_blocks, c->tune.shade_blocks, c->tune.shadow_refill, st);
  }
  { ProfScope p(c, "shade", st); launch_shade(vs, sc, fs, c->tune.shade_blocks, nl > 0, st); }
  if (atlas_wait) {
    hipError_t e = hipStreamWaitEvent(st, atlas_wait, 0);
    if (e != hipSuccess) return e;
  }
  if (any_valu) {
    ProfScope p(c, "blend_valu", st);
    launch_blend(vs, fs, st);
  }
  if (any_mma) {
    ProfScope p(c, "blend_mma", st);
    launch_blend_mma(vs, fs, c->tune.blend_blocks, c->tune.blend_rsplit, st);
  }
  return hipSuccess;
}

hipError_t enqueue_frame(irf_ctx* c, const float* rotation, hipStream_t st, hipEvent_t atlas_wait = nullptr) {
  return enqueue_frame_on(c, rotation, st, atlas_wait, volume_view(c), scratch_view(c));
}

// ---- the allocation-free frame (irf_update_probes_noalloc)
//
// Its scratch is this file-scope array: each GPU the library runs on holds
// its own copy (IRF_NOALLOC_SCRATCH_BYTES) until the process ends.  On the
// host the array's name is only a stand-in, so host code uses the device
// address that hipGetSymbolAddress gives once per device (g_noalloc_ptr),
// never the name.
static __device__ __align__(256) char g_noalloc_scratch[IRF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// Once per device, with that device current: the device address of the array.
irf_status noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(IRF_E_UNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return IRF_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_noalloc_scratch));
  if (e != hipSuccess || !p)
    return fail(IRF_E_HIP, "hipGetSymbolAddress(no-alloc scratch) failed: %s", hipGetErrorString(e));
  g_noalloc_ptr[device] = p;
  return IRF_OK;
}

// The frame's scratch carved from `base` (null: sizes only) with the sizes
// ensure_scratch gives the context's own buffers; returns the bytes used.
int64_t noalloc_layout(const irf_ctx* c, char* base, FrameScratch* fs) {
  const int64_t P = total_probes(c), R = total_rays(c);
  const int nl = c->lights.n_dir + c->lights.n_point;
  int64_t om = 0, nb = 0, wbytes = 0;
  for (int v = 0; v < c->n_vol; v++) {
    om += c->vol[v].rays;
    nb += (c->vol[v].n_probes + 1023) / 1024;
    wbytes += 256ll * c->vol[v].rays * 4;
  }
  int64_t off = 0;
  auto take = [&](int64_t bytes) -> char* {
    char* q = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return q;
  };
  FrameScratch f;
  memset(&f, 0, sizeof(f));
  f.params = (FrameParams*)take(sizeof(FrameParams));
  f.active = (int32_t*)take(sizeof(int32_t) * P);
  f.probe_pos = (float4*)take(sizeof(float4) * (P > 0 ? P : 1));
  f.block_active = (int32_t*)take(sizeof(int32_t) * (nb > 0 ? nb : 1));
  f.counters = (FrameCounters*)take(sizeof(FrameCounters));
  f.omega = (float4*)take(sizeof(float4) * om);
  f.hits = (HitRec*)take(sizeof(HitRec) * R);
  f.vis = (uint8_t*)take(R * (int64_t)(nl > 0 ? nl : 1));
  f.rays = (float4*)take(sizeof(float4) * R);
  f.shadow_tasks = (float4*)take(sizeof(float4) * kTaskRegions * task_region_cap(R, nl > 0 ? nl : 1));
  f.weights = take(wbytes > 0 ? wbytes : 16);
  f.inv_row_sum = (float*)take(sizeof(float) * 256 * (c->n_vol > 0 ? c->n_vol : 1));
  f.max_rays = R;
  f.max_slots = (int32_t)P;
  if (fs) *fs = f;
  return off;
}

// Hash of everything a captured frame bakes into its nodes.
uint64_t frame_signature(const irf_ctx* c) {
  VolumeSet vs = volume_view(c);
  FrameScratch fs = scratch_view(c);
  SceneGPU sc = scene_view(c);
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; i++) h = (h ^ b[i]) * 1099511628211ull;
  };
  mix(&vs, sizeof(vs));
  mix(&fs, sizeof(fs));
  mix(&sc, sizeof(sc));
  mix(&c->tune, sizeof(c->tune));
  // dynamic objects decide where a captured query batch runs
  const ObjectBoxes ob = boxes_view(c);
  mix(&ob, sizeof(ob));
  // a differentiable frame also writes the saved inputs
  const void* sv = c->diff ? (const void*)c->saved.p : nullptr;
  mix(&sv, sizeof(sv));
  int nl = c->lights.n_dir + c->lights.n_point;
  mix(&nl, sizeof(nl));
  return h;
}

}  // namespace

struct irf_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t params_node = nullptr;
  hipKernelNodeParams kp;
  uint64_t signature = 0;
  irf_ctx* ctx = nullptr;
};

extern "C" {

const char* irf_status_str(irf_status s) {
  switch (s) {
    case IRF_OK: return "IRF_OK";
    case IRF_E_INVALID: return "IRF_E_INVALID";
    case IRF_E_NOMEM: return "IRF_E_NOMEM";
    case IRF_E_HIP: return "IRF_E_HIP";
    case IRF_E_STATE: return "IRF_E_STATE";
    case IRF_E_UNSUPPORTED: return "IRF_E_UNSUPPORTED";
  }
  return "IRF_E_UNKNOWN";
}

const char* irf_last_error(void) { return g_err.c_str(); }

const char* irf_version(void) { return "irf 0.1 gfx950"; }

irf_status irf_create(int32_t hip_device, irf_ctx** out) {
  if (!out) return fail(IRF_E_INVALID, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) return fail(IRF_E_HIP, "no HIP device available");
  if (hip_device < 0 || hip_device >= n) return fail(IRF_E_INVALID, "device %d out of range [0, %d)", hip_device, n);
  HIP_TRY(hipSetDevice(hip_device));
  irf_status ns = noalloc_setup(hip_device);
  if (ns != IRF_OK) return ns;
  irf_ctx* c = new (std::nothrow) irf_ctx();
  if (!c) return fail(IRF_E_NOMEM, "context allocation failed");
  c->device = hip_device;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && cus > 0)
    c->tune.shadow_blocks = 16 * cus;
  memset(&c->lights, 0, sizeof(c->lights));
  for (int v = 0; v < IRF_MAX_VOLUMES; v++) c->bound[v] = false;
  *out = c;
  return IRF_OK;
}

void irf_destroy(irf_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  c->nodes.release();
  c->tris.release();
  c->albedo.release();
  c->emission.release();
  c->obj_lo.release();
  c->obj_hi.release();
  c->params.release();
  c->active.release();
  c->block_active.release();
  c->counters.release();
  c->omega.release();
  c->order.release();
  c->order_rays.clear();
  c->hits.release();
  c->vis.release();
  c->rays.release();
  c->shadow_tasks.release();
  c->stats.release();
  c->specular.release();
  c->saved.release();
  c->grad_rays.release();
  c->probe_pos.release();
  c->adj.release();
  c->weights.release();
  c->inv_row_sum.release();
  c->class_back.release();
  c->class_tf.release();
  c->reloc_keys.release();
  for (auto& r : c->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->prof_pool) (void)hipEventDestroy(e);
  delete c;
}

static irf_status validate_scene(const irf_scene_desc* d) {
  if (!d) return fail(IRF_E_INVALID, "scene desc is NULL");
  if (d->n_triangles < 0 || d->n_vertices < 0) return fail(IRF_E_INVALID, "negative counts");
  if (d->n_triangles >= (1ll << 27)) return fail(IRF_E_INVALID, "too many triangles (%lld)", (long long)d->n_triangles);
  if (d->n_materials < 1) return fail(IRF_E_INVALID, "n_materials must be >= 1");
  if (d->n_triangles > 0 && (!d->vertices || !d->indices || !d->tri_material))
    return fail(IRF_E_INVALID, "NULL geometry array");
  if (!d->albedo || !d->emission) return fail(IRF_E_INVALID, "NULL material array");
  for (int64_t i = 0; i < d->n_vertices; i++)
    if (!finite3(d->vertices + 3 * i)) return fail(IRF_E_INVALID, "vertex %lld is not finite", (long long)i);
  for (int64_t t = 0; t < d->n_triangles; t++) {
    for (int k = 0; k < 3; k++)
      if ((int64_t)d->indices[3 * t + k] >= d->n_vertices)
        return fail(IRF_E_INVALID, "triangle %lld references vertex %u >= %lld", (long long)t, d->indices[3 * t + k],
                    (long long)d->n_vertices);
    if ((int32_t)d->tri_material[t] >= d->n_materials || (int32_t)d->tri_material[t] < 0)
      return fail(IRF_E_INVALID, "triangle %lld material out of range", (long long)t);
  }
  for (int32_t m = 0; m < d->n_materials; m++)
    if (!finite3(d->albedo + 3 * m) || !finite3(d->emission + 3 * m))
      return fail(IRF_E_INVALID, "material %d is not finite", m);
  return IRF_OK;
}

irf_status irf_bvh_stats(const irf_scene_desc* d, double out[5]) {
  irf_status s = validate_scene(d);
  if (s != IRF_OK) return s;
  if (!out) return fail(IRF_E_INVALID, "out is NULL");
  std::vector<float4> nodes, tris;
  build_bvh(d->vertices, d->n_vertices, d->indices, d->n_triangles, d->tri_material, d->tri_object, nodes, tris, out);
  return IRF_OK;
}

irf_status irf_set_scene(irf_ctx* c, const irf_scene_desc* d) {
  if (!c) return fail(IRF_E_INVALID, "ctx is NULL");
  irf_status s = validate_scene(d);
  if (s != IRF_OK) return s;
  if ((s = set_device(c)) != IRF_OK) return s;
  std::vector<float4> nodes, tris;
  double st[5];
  build_bvh(d->vertices, d->n_vertices, d->indices, d->n_triangles, d->tri_material, d->tri_object, nodes, tris, st);
  if (st[4] != 1.0) return fail(IRF_E_INVALID, "BVH validation failed");
  if (st[2] > kMaxDepth) return fail(IRF_E_UNSUPPORTED, "BVH depth %g exceeds %d", st[2], kMaxDepth);
  c->frame_done = c->diff_frame = false;   // the last frame's records refer to the old scene
  // dynamic object boxes
  int32_t nobj = 0;
  if (d->tri_object)
    for (int64_t t = 0; t < d->n_triangles; t++) nobj = std::max(nobj, (int32_t)d->tri_object[t]);
  std::vector<float> lo((size_t)nobj * 3, INFINITY), hi((size_t)nobj * 3, -INFINITY);
  for (int64_t t = 0; d->tri_object && t < d->n_triangles; t++) {
    int32_t o = (int32_t)d->tri_object[t];
    if (o <= 0) continue;
    for (int k = 0; k < 3; k++)
      for (int a = 0; a < 3; a++) {
        float x = d->vertices[(size_t)d->indices[3 * t + k] * 3 + a];
        lo[(size_t)(o - 1) * 3 + a] = std::min(lo[(size_t)(o - 1) * 3 + a], x);
        hi[(size_t)(o - 1) * 3 + a] = std::max(hi[(size_t)(o - 1) * 3 + a], x);
      }
  }
  // objects with no triangles are dropped (their boxes stay empty)
  std::vector<float> blo, bhi;
  for (int32_t o = 0; o < nobj; o++)
    if (lo[(size_t)o * 3] <= hi[(size_t)o * 3])
      for (int a = 0; a < 3; a++) {
        blo.push_back(lo[(size_t)o * 3 + a]);
        bhi.push_back(hi[(size_t)o * 3 + a]);
      }
  std::vector<float4> alb((size_t)d->n_materials), emi((size_t)d->n_materials), spe((size_t)d->n_materials);
  for (int32_t m = 0; m < d->n_materials; m++) {
    alb[(size_t)m] = make_float4(d->albedo[3 * m], d->albedo[3 * m + 1], d->albedo[3 * m + 2], 0.0f);
    emi[(size_t)m] = make_float4(d->emission[3 * m], d->emission[3 * m + 1], d->emission[3 * m + 2], 0.0f);
    spe[(size_t)m] = d->specular
                         ? make_float4(d->specular[3 * m], d->specular[3 * m + 1], d->specular[3 * m + 2], 0.0f)
                         : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  HIP_TRY(hipDeviceSynchronize());
  if ((s = c->nodes.reserve(nodes.size())) != IRF_OK) return s;
  if ((s = c->tris.reserve(tris.size())) != IRF_OK) return s;
  if ((s = c->albedo.reserve(alb.size())) != IRF_OK) return s;
  if ((s = c->emission.reserve(emi.size())) != IRF_OK) return s;
  if ((s = c->specular.reserve(spe.size())) != IRF_OK) return s;
  if ((s = c->obj_lo.reserve(blo.size())) != IRF_OK) return s;
  if ((s = c->obj_hi.reserve(bhi.size())) != IRF_OK) return s;
  if (!nodes.empty()) HIP_TRY(hipMemcpy(c->nodes.p, nodes.data(), nodes.size() * sizeof(float4), hipMemcpyHostToDevice));
  if (!tris.empty()) HIP_TRY(hipMemcpy(c->tris.p, tris.data(), tris.size() * sizeof(float4), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->albedo.p, alb.data(), alb.size() * sizeof(float4), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->emission.p, emi.data(), emi.size() * sizeof(float4), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->specular.p, spe.data(), spe.size() * sizeof(float4), hipMemcpyHostToDevice));
  if (!blo.empty()) {
    HIP_TRY(hipMemcpy(c->obj_lo.p, blo.data(), blo.size() * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->obj_hi.p, bhi.data(), bhi.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  c->n_tris = (int32_t)d->n_triangles;
  c->n_nodes = (int32_t)(nodes.size() / 4);
  c->n_materials = d->n_materials;
  c->n_obj = (int32_t)(blo.size() / 3);
  for (int i = 0; i < 5; i++) c->bvh_stats[i] = st[i];
  c->has_scene = true;
  return IRF_OK;
}

irf_status irf_set_lights(irf_ctx* c, const irf_lights_desc* d) {
  if (!c || !d) return fail(IRF_E_INVALID, "NULL argument");
  if (d->n_dir < 0 || d->n_point < 0 || d->n_dir + d->n_point > IRF_MAX_LIGHTS)
    return fail(IRF_E_INVALID, "light count must be in [0, %d]", IRF_MAX_LIGHTS);
  if ((d->n_dir > 0 && (!d->dir_to_light || !d->dir_irradiance)) ||
      (d->n_point > 0 && (!d->point_pos || !d->point_intensity)))
    return fail(IRF_E_INVALID, "NULL light array");
  if (!finite3(d->sky)) return fail(IRF_E_INVALID, "sky is not finite");
  LightSet L;
  memset(&L, 0, sizeof(L));
  for (int l = 0; l < d->n_dir; l++) {
    if (!finite3(d->dir_to_light + 3 * l) || !finite3(d->dir_irradiance + 3 * l))
      return fail(IRF_E_INVALID, "directional light %d is not finite", l);
    for (int a = 0; a < 3; a++) {
      L.dir[l][a] = d->dir_to_light[3 * l + a];
      L.irr[l][a] = d->dir_irradiance[3 * l + a];
    }
  }
  for (int p = 0; p < d->n_point; p++) {
    if (!finite3(d->point_pos + 3 * p) || !finite3(d->point_intensity + 3 * p))
      return fail(IRF_E_INVALID, "point light %d is not finite", p);
    for (int a = 0; a < 3; a++) {
      L.pos[p][a] = d->point_pos[3 * p + a];
      L.irr[d->n_dir + p][a] = d->point_intensity[3 * p + a];
    }
  }
  L.n_dir = d->n_dir;
  L.n_point = d->n_point;
  for (int a = 0; a < 3; a++) L.sky[a] = d->sky[a];
  c->lights = L;
  return IRF_OK;
}

irf_status irf_validate_volume_desc(const irf_volume_desc* d) {
  if (!d) return fail(IRF_E_INVALID, "volume desc is NULL");
  int64_t P = 1;
  for (int a = 0; a < 3; a++) {
    if (d->counts[a] < 2) return fail(IRF_E_INVALID, "counts[%d] = %d must be >= 2", a, d->counts[a]);
    if (!(std::isfinite(d->spacing[a]) && d->spacing[a] > 0.0f))
      return fail(IRF_E_INVALID, "spacing[%d] must be finite and > 0", a);
    if (!std::isfinite(d->origin[a])) return fail(IRF_E_INVALID, "origin[%d] is not finite", a);
    P *= d->counts[a];
  }
  if (P > (1 << 22)) return fail(IRF_E_INVALID, "too many probes (%lld > %d)", (long long)P, 1 << 22);
  if (d->rays_per_probe < 32 || d->rays_per_probe > 1024 || d->rays_per_probe % 32)
    return fail(IRF_E_INVALID, "rays_per_probe = %d must be a multiple of 32 in [32, 1024]", d->rays_per_probe);
  if (!(d->hysteresis_irr >= 0.0f && d->hysteresis_irr <= 1.0f) ||
      !(d->hysteresis_dist >= 0.0f && d->hysteresis_dist <= 1.0f))
    return fail(IRF_E_INVALID, "hysteresis must be in [0, 1]");
  if (!(std::isfinite(d->cos_power) && d->cos_power > 0.0f)) return fail(IRF_E_INVALID, "cos_power must be > 0");
  if (!(std::isfinite(d->self_shadow_bias) && d->self_shadow_bias >= 0.0f))
    return fail(IRF_E_INVALID, "self_shadow_bias must be finite and >= 0");
  if (!std::isfinite(d->max_distance)) return fail(IRF_E_INVALID, "max_distance is not finite");
  if (d->cheb_power < 1 || d->cheb_power > 4) return fail(IRF_E_INVALID, "cheb_power must be in [1, 4]");
  if (d->atlas_dtype != IRF_ATLAS_F32 && d->atlas_dtype != IRF_ATLAS_F16)
    return fail(IRF_E_INVALID, "unknown atlas_dtype %d", d->atlas_dtype);
  if (d->blend != IRF_BLEND_F32 && d->blend != IRF_BLEND_BF16 && d->blend != IRF_BLEND_F16 &&
      d->blend != IRF_BLEND_F32_VALU)
    return fail(IRF_E_INVALID, "unknown blend %d", d->blend);
  if (!(d->irradiance_gamma == 0.0f || (d->irradiance_gamma >= 1.0f && d->irradiance_gamma <= 16.0f)))
    return fail(IRF_E_INVALID, "irradiance_gamma must be 0 (linear) or in [1, 16]");
  if (d->texel_thresholds != 0 && d->texel_thresholds != 1) return fail(IRF_E_INVALID, "texel_thresholds must be 0 or 1");
  if (d->tracking != 0 && d->tracking != 1) return fail(IRF_E_INVALID, "tracking must be 0 or 1");
  if (d->tracking)
    for (int a = 0; a < 3; a++)
      if (d->counts[a] < 5) return fail(IRF_E_INVALID, "a tracking volume needs counts >= 5 per axis");
  return IRF_OK;
}

irf_status irf_create_volume(irf_ctx* c, const irf_volume_desc* d, int32_t* volume_id) {
  if (!c || !volume_id) return fail(IRF_E_INVALID, "NULL argument");
  irf_status s = irf_validate_volume_desc(d);
  if (s != IRF_OK) return s;
  if (c->n_vol >= IRF_MAX_VOLUMES) return fail(IRF_E_INVALID, "at most %d volumes", IRF_MAX_VOLUMES);
  int64_t P = (int64_t)d->counts[0] * d->counts[1] * d->counts[2];
  if (total_probes(c) + P > (1 << 24)) return fail(IRF_E_INVALID, "too many probes in total");
  int v = c->n_vol;
  c->frame_done = c->diff_frame = false;   // the last frame did not cover this volume
  c->desc[v] = *d;
  VolumeGPU& V = c->vol[v];
  memset(&V, 0, sizeof(V));
  for (int a = 0; a < 3; a++) {
    V.origin[a] = d->origin[a];
    V.spacing[a] = d->spacing[a];
    V.inv_spacing[a] = 1.0f / d->spacing[a];
    V.counts[a] = d->counts[a];
  }
  V.n_probes = (int32_t)P;
  V.rays = d->rays_per_probe;
  V.alpha_irr = d->hysteresis_irr;
  V.alpha_dist = d->hysteresis_dist;
  V.cos_power = d->cos_power;
  V.gamma = d->irradiance_gamma == 0.0f ? 1.0f : d->irradiance_gamma;
  V.inv_gamma = 1.0f / V.gamma;
  V.half_gamma = 0.5f * V.gamma;
  V.thresholds = d->texel_thresholds;
  V.tracking = d->tracking;
  for (int a = 0; a < 3; a++) {
    V.phase[a] = 0;
    V.camera[a] = d->origin[a] + 0.5f * (float)(d->counts[a] - 1) * d->spacing[a];   // the window centre
  }
  float pi = std::floor(d->cos_power);
  V.cos_power_int = (pi == d->cos_power && pi >= 1.0f && pi <= 64.0f) ? (int32_t)pi : 0;
  V.bias = d->self_shadow_bias;
  if (d->max_distance > 0.0f) {
    V.dmax = d->max_distance;
  } else {
    double l = std::sqrt((double)d->spacing[0] * d->spacing[0] + (double)d->spacing[1] * d->spacing[1] +
                         (double)d->spacing[2] * d->spacing[2]);
    V.dmax = (float)(1.5 * l);
  }
  V.cheb_power = d->cheb_power;
  V.atlas_f16 = d->atlas_dtype == IRF_ATLAS_F16;
  V.blend = d->blend;
  V.probe_base = (int32_t)total_probes(c);
  int32_t ob = 0;
  for (int u = 0; u < v; u++) ob += c->vol[u].rays;
  V.omega_base = ob;
  int64_t wb = 0;
  for (int u = 0; u < v; u++) wb += 256ll * c->vol[u].rays * 4;
  V.weight_base = wb;
  c->bound[v] = false;
  c->n_vol = v + 1;
  *volume_id = v;
  return IRF_OK;
}

irf_status irf_volume_sizes(const irf_ctx* c, int32_t vol, irf_buffer_sizes* out) {
  if (!c || !out) return fail(IRF_E_INVALID, "NULL argument");
  if (vol < 0 || vol >= c->n_vol) return fail(IRF_E_INVALID, "volume %d does not exist", vol);
  int64_t P = c->vol[vol].n_probes;
  int64_t es = c->vol[vol].atlas_f16 ? 2 : 4;
  out->n_probes = P;
  out->irradiance_bytes = P * kIrrTexels * 4 * es;
  out->distance_bytes = P * kDistTexels * 2 * es;
  out->states_bytes = P;
  out->offsets_bytes = P * 3 * 4;
  return IRF_OK;
}

irf_status irf_bind_volume(irf_ctx* c, int32_t vol, void* irr, void* dist, uint8_t* states, const float* offsets) {
  if (!c) return fail(IRF_E_INVALID, "ctx is NULL");
  if (vol < 0 || vol >= c->n_vol) return fail(IRF_E_INVALID, "volume %d does not exist", vol);
  if (!irr || !dist || !states) return fail(IRF_E_INVALID, "NULL buffer");
  if (((uintptr_t)irr & 15) || ((uintptr_t)dist & 15) || ((uintptr_t)offsets & 3))
    return fail(IRF_E_INVALID, "buffers must be 16-byte aligned (offsets 4-byte)");
  c->vol[vol].irr = irr;
  c->vol[vol].dist = dist;
  c->vol[vol].states = states;
  c->vol[vol].offsets = offsets;
  c->bound[vol] = true;
  return IRF_OK;
}

irf_status irf_classify(irf_ctx* c, const float* rotations, int32_t K, void* stream) {
  if (!c || !rotations) return fail(IRF_E_INVALID, "NULL argument");
  if (K < 1 || K > IRF_MAX_ROTATIONS) return fail(IRF_E_INVALID, "K = %d must be in [1, %d]", K, IRF_MAX_ROTATIONS);
  for (int i = 0; i < 9 * K; i++)
    if (!std::isfinite(rotations[i])) return fail(IRF_E_INVALID, "rotation %d is not finite", i / 9);
  irf_status s = check_ready(c);
  if (s != IRF_OK) return s;
  if ((s = set_device(c)) != IRF_OK) return s;
  int64_t P = total_probes(c);
  if ((s = c->class_back.reserve((size_t)P)) != IRF_OK) return s;
  if ((s = c->class_tf.reserve((size_t)P)) != IRF_OK) return s;
  PlaneMask all;
  memset(&all, 0, sizeof(all));
  all.vol = -1;
  launch_classify(volume_view(c), scene_view(c), boxes_view(c), rotations, K, c->class_back.p, c->class_tf.p, all,
                  (hipStream_t)stream);
  return launched();
}

irf_status irf_optimize_probes(irf_ctx* c, const float* rotations, int32_t iterations, float offset_limit,
                               void* stream) {
  if (!c || !rotations) return fail(IRF_E_INVALID, "NULL argument");
  if (iterations < 1 || iterations > 64) return fail(IRF_E_INVALID, "iterations = %d must be in [1, 64]", iterations);
  if (!(offset_limit > 0.0f && offset_limit <= 0.5f)) return fail(IRF_E_INVALID, "offset_limit must be in (0, 0.5]");
  for (int i = 0; i < 9 * iterations; i++)
    if (!std::isfinite(rotations[i])) return fail(IRF_E_INVALID, "rotation %d is not finite", i / 9);
  irf_status s = check_ready(c);
  if (s != IRF_OK) return s;
  for (int v = 0; v < c->n_vol; v++)
    if (!c->vol[v].offsets) return fail(IRF_E_STATE, "volume %d has no offsets buffer bound", v);
  if ((s = set_device(c)) != IRF_OK) return s;
  int64_t P = total_probes(c);
  if ((s = c->class_back.reserve((size_t)P)) != IRF_OK) return s;
  if ((s = c->reloc_keys.reserve((size_t)(3 * P))) != IRF_OK) return s;
  for (int it = 0; it < iterations; it++)
    launch_relocate(volume_view(c), scene_view(c), rotations + 9 * it, offset_limit, c->class_back.p,
                    c->reloc_keys.p, (hipStream_t)stream);
  return launched();
}

irf_status irf_track_volume(irf_ctx* c, int32_t vol, const float* camera, const float* rotations, int32_t K,
                            int32_t* shift, void* stream) {
  if (!c || !camera || !rotations) return fail(IRF_E_INVALID, "NULL argument");
  if (vol < 0 || vol >= c->n_vol) return fail(IRF_E_INVALID, "no volume %d", vol);
  if (!c->vol[vol].tracking) return fail(IRF_E_STATE, "volume %d was not created with tracking", vol);
  if (K < 1 || K > IRF_MAX_ROTATIONS) return fail(IRF_E_INVALID, "K = %d must be in [1, %d]", K, IRF_MAX_ROTATIONS);
  for (int i = 0; i < 9 * K; i++)
    if (!std::isfinite(rotations[i])) return fail(IRF_E_INVALID, "rotation %d is not finite", i / 9);
  VolumeGPU& V = c->vol[vol];
  for (int a = 0; a < 3; a++) {
    if (!std::isfinite(camera[a])) return fail(IRF_E_INVALID, "camera is not finite");
    double center = (double)V.origin[a] + 0.5 * (double)(V.counts[a] - 1) * (double)V.spacing[a];
    if (std::fabs((double)camera[a] - center) > 1e6 * (double)V.spacing[a])
      return fail(IRF_E_INVALID, "camera more than 1e6 cells from the window");
  }
  irf_status s = check_ready(c);
  if (s != IRF_OK) return s;
  if ((s = set_device(c)) != IRF_OK) return s;
  // whole-cell shifts toward the camera while it is more than one spacing from
  // the window centre (host, double precision)
  PlaneMask m;
  memset(&m, 0, sizeof(m));
  m.vol = vol;
  int32_t k3[3];
  bool moved = false;
  for (int a = 0; a < 3; a++) {
    const double sp = (double)V.spacing[a];
    double d = (double)camera[a] - ((double)V.origin[a] + 0.5 * (double)(V.counts[a] - 1) * sp);
    int32_t k = 0;
    while (d > sp) {
      k++;
      d -= sp;
    }
    while (d < -sp) {
      k--;
      d += sp;
    }
    k3[a] = k;
    const int n = V.counts[a];
    V.origin[a] = (float)((double)V.origin[a] + (double)k * sp);
    V.phase[a] = (int32_t)((((int64_t)V.phase[a] + k) % n + n) % n);
    const int mm = k > 0 ? (k < n ? k : n) : (-k < n ? -k : n);
    if (k > 0) {
      m.lo[a] = n - mm;
      m.hi[a] = n - 1;
    } else if (k < 0) {
      m.lo[a] = 0;
      m.hi[a] = mm - 1;
    } else {
      m.lo[a] = 1;
      m.hi[a] = 0;
    }
    moved = moved || k != 0;
    V.camera[a] = camera[a];
  }
  if (shift)
    for (int a = 0; a < 3; a++) shift[a] = k3[a];
  if (moved) {
    // the entering planes start over: zero texels and offsets, classification
    if ((s = c->class_back.reserve((size_t)total_probes(c))) != IRF_OK) return s;
    if ((s = c->class_tf.reserve((size_t)total_probes(c))) != IRF_OK) return s;
    VolumeSet vs = volume_view(c);
    launch_track_reset(vs, m, (hipStream_t)stream);
    launch_classify(vs, scene_view(c), boxes_view(c), rotations, K, c->class_back.p, c->class_tf.p, m,
                    (hipStream_t)stream);
  }
  return launched();
}

irf_status irf_volume_window(const irf_ctx* c, int32_t vol, float origin[3], int32_t phase[3], float camera[3]) {
  if (!c || !origin || !phase || !camera) return fail(IRF_E_INVALID, "NULL argument");
  if (vol < 0 || vol >= c->n_vol) return fail(IRF_E_INVALID, "no volume %d", vol);
  for (int a = 0; a < 3; a++) {
    origin[a] = c->vol[vol].origin[a];
    phase[a] = c->vol[vol].phase[a];
    camera[a] = c->vol[vol].camera[a];
  }
  return IRF_OK;
}

irf_status irf_update_probes_after(irf_ctx* c, const float* rotation, void* stream, void* atlas_event) {
  if (!c || !rotation) return fail(IRF_E_INVALID, "NULL argument");
  for (int i = 0; i < 9; i++)
    if (!std::isfinite(rotation[i])) return fail(IRF_E_INVALID, "rotation is not finite");
  irf_status s = check_ready(c);
  if (s != IRF_OK) return s;
  if ((s = set_device(c)) != IRF_OK) return s;
  if ((s = ensure_scratch(c)) != IRF_OK) return s;
  if (atlas_event) {
    // reject a bad event before any of the frame is enqueued
    hipError_t q = hipEventQuery((hipEvent_t)atlas_event);
    if (q != hipSuccess && q != hipErrorNotReady)
      return fail(IRF_E_INVALID, "atlas_event is not a usable event: %s", hipGetErrorString(q));
  }
  hipError_t e = enqueue_frame(c, rotation, (hipStream_t)stream, (hipEvent_t)atlas_event);
  if (e != hipSuccess) return fail(IRF_E_HIP, "waiting on the atlas event: %s", hipGetErrorString(e));
  c->frame_done = true;
  c->diff_frame = c->diff;
  return launched();
}

irf_status irf_update_probes(irf_ctx* c, const float* rotation, void* stream) {
  return irf_update_probes_after(c, rotation, stream, nullptr);
}

irf_status irf_update_probes_query(irf_ctx* c, const float* rotation, const float* pos, const float* nrm,
                                   const float* view, int64_t n, float* out, void* stream) {
  if (!c || !rotation) return fail(IRF_E_INVALID, "NULL argument");
  if (n < 0) return fail(IRF_E_INVALID, "n < 0");
  if (n > 0 && (!pos || !nrm || !view || !out)) return fail(IRF_E_INVALID, "NULL array");
  for (int i = 0; i < 9; i++)
    if (!std::isfinite(rotation[i])) return fail(IRF_E_INVALID, "rotation is not finite");
  irf_status s = check_ready(c);
  if (s != IRF_OK) return s;
  if ((s = set_device(c)) != IRF_OK) return s;
  if ((s = ensure_scratch(c)) != IRF_OK) return s;
  const QueryBatch qb = {pos, nrm, view, out, 0, n};
  hipError_t e = enqueue_frame_on(c, rotation, (hipStream_t)stream, nullptr, volume_view(c), scratch_view(c), &qb);
  if (e != hipSuccess) return fail(IRF_E_HIP, "enqueueing the frame: %s", hipGetErrorString(e));
  c->frame_done = true;
  c->diff_frame = c->diff;
  return launched();
}

irf_status irf_update_probes_noalloc(irf_ctx* c, const float* rotation, void* stream) {
  if (!c || !rotation) return fail(IRF_E_INVALID, "NULL argument");
  for (int i = 0; i < 9; i++)
    if (!std::isfinite(rotation[i])) return fail(IRF_E_INVALID, "rotation is not finite");
  irf_status s = check_ready(c);
  if (s != IRF_OK) return s;
  if (c->diff)
    return fail(IRF_E_UNSUPPORTED, "the no-alloc frame does not save a differentiable frame's inputs");
  const int64_t need = noalloc_layout(c, nullptr, nullptr);
  if (need > IRF_NOALLOC_SCRATCH_BYTES)
    return fail(IRF_E_UNSUPPORTED, "the frame needs %lld bytes of scratch; the no-alloc scratch holds %lld",
                (long long)need, (long long)IRF_NOALLOC_SCRATCH_BYTES);
  if ((s = set_device(c)) != IRF_OK) return s;
  void* base = c->device >= 0 && c->device < kMaxDevices ? g_noalloc_ptr[c->device] : nullptr;
  if (!base) return fail(IRF_E_STATE, "no-alloc scratch not set up on device %d", c->device);
  FrameScratch fs;
  noalloc_layout(c, (char*)base, &fs);
  // the coherent ray order is a library-owned table: traced in index order
  // here (only the lane a ray runs on changes, no result)
  VolumeSet vs = volume_view(c);
  for (int v = 0; v < vs.n; v++) vs.v[v].order = nullptr;
  const bool prof = c->prof;
  c->prof = false;   // kernel timing would create events
  hipError_t e = enqueue_frame_on(c, rotation, (hipStream_t)stream, nullptr, vs, fs);
  c->prof = prof;
  if (e != hipSuccess) return fail(IRF_E_HIP, "enqueueing the frame: %s", hipGetErrorString(e));
  // the context's own scratch does not hold this frame: no records or stats
  c->frame_done = false;
  c->diff_frame = false;
  return launched();
}

irf_status irf_query_irradiance(irf_ctx* c, const float* pos, const float* nrm, const float* view, int64_t n,
                                float* out, void* stream) {
  if (!c) return fail(IRF_E_INVALID, "ctx is NULL");
  if (n < 0) return fail(IRF_E_INVALID, "n < 0");
  if (n == 0) return IRF_OK;
  if (!pos || !nrm || !view || !out) return fail(IRF_E_INVALID, "NULL array");
  if (c->n_vol == 0) return fail(IRF_E_STATE, "no volume");
  for (int v = 0; v < c->n_vol; v++)
    if (!c->bound[v]) return fail(IRF_E_STATE, "volume %d has no bound buffers", v);
  irf_status s = set_device(c);
  if (s != IRF_OK) return s;
  {
    ProfScope p(c, "query", (hipStream_t)stream);
    launch_query(volume_view(c), pos, nrm, view, n, out, (hipStream_t)stream);
  }
  return launched();
}

irf_status irf_ray_records(irf_ctx* c, int32_t vol, irf_ray_record* out, int64_t capacity, int64_t* count,
                           void* stream) {
  if (!c || !count) return fail(IRF_E_INVALID, "NULL argument");
  if (vol < 0 || vol >= c->n_vol) return fail(IRF_E_INVALID, "volume %d does not exist", vol);
  if (!c->frame_done) return fail(IRF_E_STATE, "no update frame has run");
  irf_status s = set_device(c);
  if (s != IRF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  FrameCounters C;
  HIP_TRY(hipMemcpyAsync(&C, c->counters.p, sizeof(C), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  int64_t n = C.ray_base[vol + 1] - C.ray_base[vol];
  *count = n;
  if (!out || capacity <= 0) return IRF_OK;
  launch_records(volume_view(c), vol, scene_view(c), scratch_view(c), c->lights.n_dir + c->lights.n_point, out,
                 n < capacity ? n : capacity, st);
  return launched();
}

irf_status irf_frame_stats(irf_ctx* c, int64_t out[4], void* stream) {
  if (!c || !out) return fail(IRF_E_INVALID, "NULL argument");
  if (!c->frame_done) return fail(IRF_E_STATE, "no update frame has run");
  irf_status s = set_device(c);
  if (s != IRF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  launch_frame_stats(volume_view(c), scene_view(c), scratch_view(c), c->stats.p, st);
  if ((s = launched()) != IRF_OK) return s;
  FrameCounters C;
  unsigned long long k[4];
  HIP_TRY(hipMemcpyAsync(&C, c->counters.p, sizeof(C), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(k, c->stats.p, sizeof(k), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  out[0] = C.slot_base[c->n_vol];
  out[1] = C.ray_base[c->n_vol];
  out[2] = c->lights.n_dir + c->lights.n_point > 0 ? (int64_t)k[0] : 0;
  out[3] = (int64_t)k[1];
  return IRF_OK;
}

irf_status irf_traversal_stats(irf_ctx* c, int64_t out[4], void* stream) {
  if (!c || !out) return fail(IRF_E_INVALID, "NULL argument");
  if (!c->frame_done) return fail(IRF_E_STATE, "no update frame has run");
  irf_status s = set_device(c);
  if (s != IRF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  launch_traversal_stats(volume_view(c), scene_view(c), c->lights.n_dir + c->lights.n_point, scratch_view(c),
                         c->stats.p, st);
  if ((s = launched()) != IRF_OK) return s;
  unsigned long long k[4];
  HIP_TRY(hipMemcpyAsync(k, c->stats.p, sizeof(k), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int i = 0; i < 4; i++) out[i] = (int64_t)k[i];
  return IRF_OK;
}

irf_status irf_set_tuning(irf_ctx* c, const irf_tuning* t) {
  if (!c || !t) return fail(IRF_E_INVALID, "NULL argument");
  if (t->trace_blocks < 0 || t->shadow_blocks < 0 || t->shade_blocks < 0 || t->blend_blocks < 0)
    return fail(IRF_E_INVALID, "tuning values must be >= 0");
  if (t->shadow_refill < 0 || t->shadow_refill > 64)
    return fail(IRF_E_INVALID, "shadow_refill must be in [0, 64]");
  if (t->blend_rsplit != 0 && t->blend_rsplit != 1 && t->blend_rsplit != 2 && t->blend_rsplit != 4)
    return fail(IRF_E_INVALID, "blend_rsplit must be 0, 1, 2 or 4");
  if (t->query_shadow < 0 || t->query_shadow > 1000) return fail(IRF_E_INVALID, "query_shadow must be in [0, 1000]");
  c->tune.trace_blocks = t->trace_blocks;
  c->tune.shadow_blocks = t->shadow_blocks;
  c->tune.shade_blocks = t->shade_blocks;
  c->tune.blend_blocks = t->blend_blocks;
  c->tune.shadow_refill = t->shadow_refill;
  c->tune.blend_rsplit = t->blend_rsplit;
  c->tune.query_shadow = t->query_shadow;
  return IRF_OK;
}

irf_status irf_get_tuning(const irf_ctx* c, irf_tuning* t) {
  if (!c || !t) return fail(IRF_E_INVALID, "NULL argument");
  t->trace_blocks = c->tune.trace_blocks;
  t->shadow_blocks = c->tune.shadow_blocks;
  t->shade_blocks = c->tune.shade_blocks;
  t->blend_blocks = c->tune.blend_blocks;
  t->shadow_refill = c->tune.shadow_refill;
  t->blend_rsplit = c->tune.blend_rsplit;
  t->query_shadow = c->tune.query_shadow;
  return IRF_OK;
}

// The frame (with a query batch when qb is given) captured on `stream`.
irf_status capture_frame(irf_ctx* c, void* stream, const QueryBatch* qb, irf_graph** out) {
  if (!c || !out) return fail(IRF_E_INVALID, "NULL argument");
  *out = nullptr;
  if (!stream) return fail(IRF_E_INVALID, "capture needs a stream other than the null stream");
  irf_status s = check_ready(c);
  if (s != IRF_OK) return s;
  if ((s = set_device(c)) != IRF_OK) return s;
  if ((s = ensure_scratch(c)) != IRF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const float identity[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  const bool prof = c->prof;
  c->prof = false;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    c->prof = prof;
    return fail(IRF_E_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  // the capture is always ended, and the graph destroyed on any failure
  const hipError_t qe = enqueue_frame_on(c, identity, st, nullptr, volume_view(c), scratch_view(c), qb);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(st, &graph);
  c->prof = prof;
  if (e != hipSuccess) return fail(IRF_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  if (qe != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(IRF_E_HIP, "capturing the frame: %s", hipGetErrorString(qe));
  }
  size_t n = 0;
  std::vector<hipGraphNode_t> nodes;
  e = hipGraphGetNodes(graph, nullptr, &n);
  if (e == hipSuccess && n) {
    nodes.resize(n);
    e = hipGraphGetNodes(graph, nodes.data(), &n);
  }
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(IRF_E_HIP, "hipGraphGetNodes: %s", hipGetErrorString(e));
  }
  irf_graph* g = new irf_graph();
  g->graph = graph;
  g->ctx = c;
  for (auto node : nodes) {
    hipGraphNodeType type;
    if (hipGraphNodeGetType(node, &type) != hipSuccess || type != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams kp;
    if (hipGraphKernelNodeGetParams(node, &kp) != hipSuccess) continue;
    if (kp.func == frame_begin_kernel()) {
      g->params_node = node;
      g->kp = kp;
    }
  }
  if (!g->params_node) {
    (void)hipGraphDestroy(graph);
    delete g;
    return fail(IRF_E_HIP, "captured frame has no parameter node");
  }
  e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    delete g;
    return fail(IRF_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  // the executable graph goes to the device now: otherwise its first launch
  // pays the upload (about 0.8 ms for the city frame, measured)
  e = hipGraphUpload(g->exec, st);
  if (e != hipSuccess) {
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(graph);
    delete g;
    return fail(IRF_E_HIP, "hipGraphUpload: %s", hipGetErrorString(e));
  }
  g->signature = frame_signature(c);
  *out = g;
  return IRF_OK;
}

irf_status irf_graph_capture(irf_ctx* c, void* stream, irf_graph** out) {
  return capture_frame(c, stream, nullptr, out);
}

irf_status irf_graph_capture_query(irf_ctx* c, void* stream, const float* pos, const float* nrm, const float* view,
                                   int64_t n, float* out_rgb, irf_graph** out) {
  if (!c || !out) return fail(IRF_E_INVALID, "NULL argument");
  *out = nullptr;
  if (n < 0) return fail(IRF_E_INVALID, "n < 0");
  if (n > 0 && (!pos || !nrm || !view || !out_rgb)) return fail(IRF_E_INVALID, "NULL array");
  const QueryBatch qb = {pos, nrm, view, out_rgb, 0, n};
  return capture_frame(c, stream, &qb, out);
}

irf_status irf_graph_launch(irf_ctx* c, irf_graph* g, const float* rotation, void* stream) {
  if (!c || !g || !rotation) return fail(IRF_E_INVALID, "NULL argument");
  if (g->ctx != c) return fail(IRF_E_INVALID, "graph belongs to another context");
  for (int i = 0; i < 9; i++)
    if (!std::isfinite(rotation[i])) return fail(IRF_E_INVALID, "rotation is not finite");
  if (frame_signature(c) != g->signature)
    return fail(IRF_E_STATE, "scene, volumes, buffers, light count or tuning changed since capture: capture again");
  irf_status s = set_device(c);
  if (s != IRF_OK) return s;
  FrameParams fp;
  for (int i = 0; i < 9; i++) fp.R[i] = rotation[i];
  fp.L = c->lights;
  bool any_mma = false;
  for (int v = 0; v < c->n_vol; v++) any_mma = any_mma || c->vol[v].blend != IRF_BLEND_F32_VALU;
  FrameBegin fb = make_frame_begin(fp, volume_view(c), boxes_view(c), scratch_view(c), any_mma);
  void* args[1] = {&fb};
  hipKernelNodeParams kp = g->kp;
  kp.kernelParams = args;
  kp.extra = nullptr;
  HIP_TRY(hipGraphExecKernelNodeSetParams(g->exec, g->params_node, &kp));
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
  c->frame_done = true;
  c->diff_frame = c->diff;   // the signature pins the mode to the capture's
  return IRF_OK;
}

void irf_graph_destroy(irf_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

irf_status irf_trace_glossy(irf_ctx* c, const float* pos, const float* nrm, const float* view, int64_t n,
                            float* out_rgb, irf_ray_record* records, void* stream) {
  if (!c) return fail(IRF_E_INVALID, "ctx is NULL");
  if (n < 0) return fail(IRF_E_INVALID, "n < 0");
  if (n == 0) return IRF_OK;
  if (!pos || !nrm || !view || !out_rgb) return fail(IRF_E_INVALID, "NULL array");
  irf_status s = check_ready(c);
  if (s != IRF_OK) return s;
  if ((s = set_device(c)) != IRF_OK) return s;
  launch_glossy(volume_view(c), scene_view(c), c->lights, pos, nrm, view, n, out_rgb, records, (hipStream_t)stream);
  return launched();
}

irf_status irf_set_differentiable(irf_ctx* c, int32_t enable) {
  if (!c) return fail(IRF_E_INVALID, "ctx is NULL");
  c->diff = enable != 0;
  c->diff_frame = false;   // a backward needs a frame run in this mode
  return IRF_OK;
}

irf_status irf_set_emission(irf_ctx* c, const float* emission, void* stream) {
  if (!c || !emission) return fail(IRF_E_INVALID, "NULL argument");
  if (!c->has_scene) return fail(IRF_E_STATE, "no scene");
  irf_status s = set_device(c);
  if (s != IRF_OK) return s;
  launch_set_emission(emission, c->emission.p, c->n_materials, (hipStream_t)stream);
  return launched();
}

static irf_status grad_set(const irf_ctx* c, float* const* irr, float* const* dist, GradSet& G) {
  memset(&G, 0, sizeof(G));
  if (!irr || !dist) return fail(IRF_E_INVALID, "NULL gradient array");
  for (int v = 0; v < c->n_vol; v++) {
    if (c->vol[v].atlas_f16) return fail(IRF_E_UNSUPPORTED, "gradients need float32 atlases");
    if (c->vol[v].gamma != 1.0f || c->vol[v].thresholds)
      return fail(IRF_E_UNSUPPORTED, "gradients need linear irradiance texels without per-texel thresholds");
    if (!irr[v] || !dist[v]) return fail(IRF_E_INVALID, "NULL gradient buffer for volume %d", v);
    G.irr[v] = irr[v];
    G.dist[v] = dist[v];
  }
  return IRF_OK;
}

// Terms of one batch of the adjoint's gradient sums: 2^22 (168 MB of terms,
// 48 MB of keys and sorted order); a frame's rays or a query's points go through
// in batches of that many terms.
constexpr int64_t kAdjTerms = 1ll << 22;

static irf_status adjoint_scratch(irf_ctx* c, AdjointScratch& A) {
  int64_t K = c->n_materials > 0 ? c->n_materials : 0;
  for (int v = 0; v < c->n_vol; v++) K += c->vol[v].n_probes;
  if (K < 1) K = 1;
  const int64_t slots = adjoint_partial_slots(kAdjTerms);
  const size_t sort_bytes = adjoint_sort_bytes(kAdjTerms);
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t T4 = up(4 * (size_t)kAdjTerms), K4 = up(4 * (size_t)(K + 1));
  const size_t sizes[] = {up(40 * (size_t)kAdjTerms), T4, T4, T4, K4, K4, K4, K4,
                          up(adjoint_slot_bytes() * (size_t)slots),
                          up(sizeof(float) * (size_t)adjoint_norms_per_volume() * IRF_MAX_VOLUMES), up(sort_bytes)};
  constexpr int kParts = sizeof(sizes) / sizeof(sizes[0]);
  size_t total = 0;
  for (size_t b : sizes) total += b;
  irf_status s = c->adj.reserve(total);
  if (s != IRF_OK) return s;
  char* q = c->adj.p;
  void* part[kParts];
  for (int i = 0; i < kParts; i++) {
    part[i] = q;
    q += sizes[i];
  }
  A.terms = part[0];
  A.keys[0] = (uint32_t*)part[1];
  A.keys[1] = (uint32_t*)part[2];
  A.idx = (uint32_t*)part[3];
  A.seg_start = (uint32_t*)part[4];
  A.seg_end = (uint32_t*)part[5];
  A.offs = (uint32_t*)part[6];
  A.poffs = (uint32_t*)part[7];
  A.partial = (float*)part[8];
  A.norms = (float*)part[9];
  A.sort_temp = part[10];
  A.sort_bytes = sort_bytes;
  A.max_terms = kAdjTerms;
  A.max_partial = slots;
  return IRF_OK;
}

irf_status irf_query_backward(irf_ctx* c, const float* pos, const float* nrm, const float* view, int64_t n,
                              const float* grad_out, float* const* grad_irr, float* const* grad_dist, void* stream) {
  if (!c) return fail(IRF_E_INVALID, "ctx is NULL");
  if (n < 0) return fail(IRF_E_INVALID, "n < 0");
  if (n == 0) return IRF_OK;
  if (!pos || !nrm || !view || !grad_out) return fail(IRF_E_INVALID, "NULL array");
  irf_status s = check_ready(c);
  if (s != IRF_OK) return s;
  GradSet G;
  if ((s = grad_set(c, grad_irr, grad_dist, G)) != IRF_OK) return s;
  if ((s = set_device(c)) != IRF_OK) return s;
  AdjointScratch A;
  if ((s = adjoint_scratch(c, A)) != IRF_OK) return s;
  HIP_TRY(launch_query_backward(volume_view(c), pos, nrm, view, n, grad_out, G, A, (hipStream_t)stream));
  return launched();
}

irf_status irf_update_backward(irf_ctx* c, float* const* g_new_irr, float* const* g_new_dist, float* const* g_prev_irr,
                               float* const* g_prev_dist, float* g_emission, void* stream) {
  if (!c || !g_emission) return fail(IRF_E_INVALID, "NULL argument");
  if (!c->diff_frame) return fail(IRF_E_STATE, "no frame was run with irf_set_differentiable(ctx, 1)");
  irf_status s;
  GradSet Gn, Gp;
  if ((s = grad_set(c, g_new_irr, g_new_dist, Gn)) != IRF_OK) return s;
  if ((s = grad_set(c, g_prev_irr, g_prev_dist, Gp)) != IRF_OK) return s;
  if ((s = set_device(c)) != IRF_OK) return s;
  VolumeSet prev = volume_view(c);
  for (int v = 0; v < c->n_vol; v++) {
    prev.v[v].irr = c->saved.p + c->saved_irr[v];
    prev.v[v].dist = c->saved.p + c->saved_dist[v];
    prev.v[v].states = (uint8_t*)(c->saved.p + c->saved_states[v]);
  }
  AdjointScratch A;
  if ((s = adjoint_scratch(c, A)) != IRF_OK) return s;
  // the frame's ray count bounds the batches (most probes of a sparse frame
  // trace nothing)
  FrameCounters fc;
  HIP_TRY(hipMemcpyAsync(&fc, c->counters.p, sizeof(fc), hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  HIP_TRY(launch_update_backward(prev, scene_view(c), scratch_view(c), Gn, Gp, g_emission, c->n_materials,
                                 fc.ray_base[c->n_vol], A, (hipStream_t)stream));
  return launched();
}

irf_status irf_profile_enable(irf_ctx* c, int32_t enable) {
  if (!c) return fail(IRF_E_INVALID, "ctx is NULL");
  c->prof = enable != 0;
  return IRF_OK;
}

irf_status irf_profile_read(irf_ctx* c, irf_kernel_time* out, int32_t capacity, int32_t* count, int32_t reset) {
  if (!c || !count) return fail(IRF_E_INVALID, "NULL argument");
  irf_status s = set_device(c);
  if (s != IRF_OK) return s;
  for (auto& r : c->prof_pending) {
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    auto& acc = c->prof_acc[r.name];
    acc.first += 1;
    acc.second += ms;
    c->prof_pool.push_back(r.a);
    c->prof_pool.push_back(r.b);
  }
  c->prof_pending.clear();
  int32_t n = 0;
  for (auto& kv : c->prof_acc) {
    if (out && n < capacity) {
      memset(out[n].name, 0, sizeof(out[n].name));
      strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
      out[n].launches = kv.second.first;
      out[n].total_ms = kv.second.second;
    }
    n++;
  }
  *count = n;
  if (reset) c->prof_acc.clear();
  return IRF_OK;
}

}  // extern "C"
