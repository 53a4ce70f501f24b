// Per-frame bookkeeping and the vector-ALU blend of the probe update, plus
// the query kernel.
//
//  k_directions     rotated spherical-Fibonacci ray directions of the frame
//                   (one rotation shared by every probe of every volume)
//  k_state_compact  per-frame state step (dynamic-object wake/sleep) and the
//                   list of active probes, packed across volumes
//  k_blend_f32      Eq. U per texel as a normalised weighted average with
//                   hysteresis; one workgroup per active probe with the
//                   probe's rays in LDS (the paper's coherent compute-shader
//                   update), border texels written by their source texel
//  k_query          E(X, n, w_o) for a batch of points
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace irf {

__device__ __forceinline__ float3 sf_dir(int i, int n, const float* R) {
  // frac(i * golden ratio) exactly, from the 0.64 fixed-point golden ratio
  uint64_t fr = (uint64_t)i * 0x9E3779B97F4A7C15ull;
  float f = (float)(fr >> 40) * 0x1p-24f;
  float t = (float)(2 * i + 1) / (float)n;
  float z = 1.0f - t;
  float rr = sqrtf(t * (2.0f - t));
  float sn, cs;
  sincospif(2.0f * f, &sn, &cs);
  float3 p = f3(rr * cs, rr * sn, z);
  return f3(fmaf(R[0], p.x, fmaf(R[1], p.y, R[2] * p.z)), fmaf(R[3], p.x, fmaf(R[4], p.y, R[5] * p.z)),
            fmaf(R[6], p.x, fmaf(R[7], p.y, R[8] * p.z)));
}

// The frame's parameters (rotation, lights) are kernel arguments of this one
// node, so a captured frame is re-launched with new ones by updating it.
__global__ void k_set_params(FrameParams p, FrameParams* dst) {
  if (threadIdx.x == 0) *dst = p;
}

__global__ void k_directions(VolumeSet vs, FrameScratch fs) {
  int v = blockIdx.y;
  if (v >= vs.n) return;
  const VolumeGPU& V = vs.v[v];
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= V.rays) return;
  float3 w = sf_dir(r, V.rays, fs.params->R);
  fs.omega[V.omega_base + r] = make_float4(w.x, w.y, w.z, 0.0f);
}

__device__ __forceinline__ bool active_state(uint8_t s) {
  return s == IRF_NEWLY_AWAKE || s == IRF_NEWLY_VIGILANT || s == IRF_AWAKE || s == IRF_VIGILANT;
}

__device__ __forceinline__ bool near_dynamic(const VolumeGPU& V, ObjectBoxes ob, float3 P) {
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

constexpr int kCompactBlock = 1024;

// Workgroups of volume v: [A.block_base[v], A.block_base[v+1]), each covering
// kCompactBlock consecutive probes of that volume only.
struct CompactArgs {
  int32_t block_base[IRF_MAX_VOLUMES + 1];
};

__device__ __forceinline__ int compact_volume(const CompactArgs& A, int nvol, int b) {
  int v = 0;
  while (v + 1 < nvol && b >= A.block_base[v + 1]) v++;
  return v;
}

// Pass 1: state step (dynamic-object wake/sleep) and the number of active
// probes of every workgroup.
__global__ __launch_bounds__(kCompactBlock) void k_state_count(VolumeSet vs, ObjectBoxes ob, CompactArgs A,
                                                                FrameScratch fs) {
  __shared__ int wave_tot[kCompactBlock / 64];
  const int b = blockIdx.x;
  const int v = compact_volume(A, vs.n, b);
  const VolumeGPU& V = vs.v[v];
  const int q = (b - A.block_base[v]) * kCompactBlock + threadIdx.x;
  bool act = false;
  if (q < V.n_probes) {
    uint8_t st = V.states[q];
    if (ob.n > 0 && (st == IRF_SLEEPING || st == IRF_AWAKE)) {
      bool near = near_dynamic(V, ob, probe_position(V, q));
      uint8_t ns = st;
      if (st == IRF_SLEEPING && near) ns = IRF_NEWLY_AWAKE;
      if (st == IRF_AWAKE && !near) ns = IRF_SLEEPING;
      if (ns != st) V.states[q] = ns;
      st = ns;
    }
    act = active_state(st);
  }
  unsigned long long m = __ballot(act);
  if ((threadIdx.x & 63) == 0) wave_tot[threadIdx.x >> 6] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kCompactBlock / 64; w++) t += wave_tot[w];
    fs.block_active[b] = t;
  }
}

// Pass 2: ordered scatter of the active list (ascending probe index within a
// volume, volumes in order) and the per-volume slot and ray bases.
__global__ __launch_bounds__(kCompactBlock) void k_state_scatter(VolumeSet vs, CompactArgs A, FrameScratch fs) {
  __shared__ int wave_off[kCompactBlock / 64];
  __shared__ int s_base;
  const int b = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int v = compact_volume(A, vs.n, b);
  const VolumeGPU& V = vs.v[v];
  // offset of this workgroup: active probes of all earlier workgroups
  if (wave == 0) {
    int part = 0;
    for (int i = lane; i < b; i += 64) part += fs.block_active[i];
    for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off);
    if (lane == 0) s_base = part;
  }
  const int q = (b - A.block_base[v]) * kCompactBlock + threadIdx.x;
  const bool act = q < V.n_probes && active_state(V.states[q]);
  unsigned long long m = __ballot(act);
  if (lane == 0) wave_off[wave] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < kCompactBlock / 64; w++) {
      int t = wave_off[w];
      wave_off[w] = acc;
      acc += t;
    }
  }
  __syncthreads();
  if (act) {
    const int slot = s_base + wave_off[wave] + __popcll(m & ((1ull << lane) - 1ull));
    fs.active[slot] = V.probe_base + q;
    const float3 P = probe_position(V, q);
    fs.probe_pos[slot] = make_float4(P.x, P.y, P.z, 0.0f);
  }
  if (b == 0 && threadIdx.x == 0) {
    FrameCounters C;
    int slot = 0;
    int64_t rays = 0;
    for (int u = 0; u < vs.n; u++) {
      C.slot_base[u] = slot;
      C.ray_base[u] = rays;
      int cnt = 0;
      for (int i = A.block_base[u]; i < A.block_base[u + 1]; i++) cnt += fs.block_active[i];
      slot += cnt;
      rays += (int64_t)cnt * vs.v[u].rays;
    }
    C.slot_base[vs.n] = slot;
    C.ray_base[vs.n] = rays;
    C.shadow_total = 0;
    *fs.counters = C;
  }
}

// ---- blend (vector ALU, float32)

constexpr int kBlendBlock = 256;
constexpr int kDistInterior = (kDistTile - 2) * (kDistTile - 2);   // 196
constexpr int kIrrInterior = (kIrrTile - 2) * (kIrrTile - 2);      // 36

// Writes value to interior cell (x, y) of an M-tile and to every border cell
// that repeats it.
template <int M, typename F>
__device__ __forceinline__ void store_with_border(int x, int y, F store) {
  constexpr int k = M - 2;
  store(x, y);
  if (y == 1) store(k + 1 - x, 0);
  if (y == k) store(k + 1 - x, k + 1);
  if (x == 1) store(0, k + 1 - y);
  if (x == k) store(k + 1, k + 1 - y);
  if (x == k && y == k) store(0, 0);
  if (x == 1 && y == k) store(k + 1, 0);
  if (x == k && y == 1) store(0, k + 1);
  if (x == 1 && y == 1) store(k + 1, k + 1);
}

__global__ __launch_bounds__(kBlendBlock) void k_blend_f32(VolumeSet vs, FrameScratch fs) {
  __shared__ float4 s_ray[1024];
  __shared__ float4 s_om[1024];
  const FrameCounters& C = *fs.counters;
  int gslot = blockIdx.x;
  if (gslot >= C.slot_base[vs.n]) return;
  int v = 0;
  while (v + 1 < vs.n && gslot >= C.slot_base[v + 1]) v++;
  const VolumeGPU& V = vs.v[v];
  if (V.blend != IRF_BLEND_F32_VALU) return;
  int slot = gslot - C.slot_base[v];
  int q = fs.active[gslot] - V.probe_base;
  const int N = V.rays;
  const float4* R = fs.rays + C.ray_base[v] + (int64_t)slot * N;
  for (int i = threadIdx.x; i < N; i += kBlendBlock) {
    s_ray[i] = R[i];
    s_om[i] = fs.omega[V.omega_base + i];
  }
  uint8_t st = V.states[q];
  bool fresh = st == IRF_NEWLY_AWAKE || st == IRF_NEWLY_VIGILANT;
  __syncthreads();
  int t = threadIdx.x;
  if (t < kDistInterior) {
    int x = t % (kDistTile - 2) + 1, y = t / (kDistTile - 2) + 1;
    float3 n = texel_direction<kDistTile>(x, y);
    float W = 0.0f, m1 = 0.0f, m2 = 0.0f;
    for (int r = 0; r < N; r++) {
      float4 o = s_om[r];
      float c = fmaf(n.x, o.x, fmaf(n.y, o.y, n.z * o.z));
      if (c > 0.0f) {
        float w = pow_weight(c, V);
        float d = s_ray[r].w;
        W += w;
        m1 = fmaf(w, d, m1);
        m2 = fmaf(w * d, d, m2);
      }
    }
    if (W > 0.0f) {
      float a = fresh ? 0.0f : V.alpha_dist;
      int idx = q * kDistTexels + y * kDistTile + x;
      float2 old = load_dist(V, idx);
      float n1 = m1 / W, n2 = m2 / W;
      float2 val = make_float2(a * old.x + (1.0f - a) * n1, a * old.y + (1.0f - a) * n2);
      store_with_border<kDistTile>(x, y, [&](int xx, int yy) {
        int j = q * kDistTexels + yy * kDistTile + xx;
        if (V.atlas_f16) {
          h2 h;
          h.x = (_Float16)val.x;
          h.y = (_Float16)val.y;
          ((h2*)V.dist)[j] = h;
        } else {
          ((float2*)V.dist)[j] = val;
        }
      });
    }
  } else if (t < kDistInterior + kIrrInterior) {
    int u = t - kDistInterior;
    int x = u % (kIrrTile - 2) + 1, y = u / (kIrrTile - 2) + 1;
    float3 n = texel_direction<kIrrTile>(x, y);
    float W = 0.0f;
    float3 acc = f3(0.0f, 0.0f, 0.0f);
    for (int r = 0; r < N; r++) {
      float4 o = s_om[r];
      float c = fmaf(n.x, o.x, fmaf(n.y, o.y, n.z * o.z));
      if (c > 0.0f) {
        float4 L = s_ray[r];
        W += c;
        acc = f3(fmaf(c, L.x, acc.x), fmaf(c, L.y, acc.y), fmaf(c, L.z, acc.z));
      }
    }
    if (W > 0.0f) {
      float a = fresh ? 0.0f : V.alpha_irr;
      int idx = q * kIrrTexels + y * kIrrTile + x;
      float3 old = load_irr(V, idx);
      float iw = 1.0f / W;
      float3 val = irr_texel_update(V, a, old, f3(acc.x * iw, acc.y * iw, acc.z * iw));
      store_with_border<kIrrTile>(x, y, [&](int xx, int yy) {
        int j = q * kIrrTexels + yy * kIrrTile + xx;
        if (V.atlas_f16) {
          h4 h;
          h.x = (_Float16)val.x;
          h.y = (_Float16)val.y;
          h.z = (_Float16)val.z;
          h.w = (_Float16)0.0f;
          ((h4*)V.irr)[j] = h;
        } else {
          ((float4*)V.irr)[j] = make_float4(val.x, val.y, val.z, 0.0f);
        }
      });
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && fresh) V.states[q] = st == IRF_NEWLY_AWAKE ? IRF_AWAKE : IRF_VIGILANT;
}

// ---- query

constexpr int kQueryBlock = 256;

__global__ __launch_bounds__(kQueryBlock) void k_query(VolumeSet vs, const float* __restrict__ pos,
                                                      const float* __restrict__ nrm, const float* __restrict__ view,
                                                      int64_t n, float* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * kQueryBlock + threadIdx.x;
  if (i >= n) return;
  float3 X = f3(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
  float3 N = f3(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]);
  float3 Wo = f3(view[3 * i], view[3 * i + 1], view[3 * i + 2]);
  float3 E = query_irradiance(vs, X, N, Wo);
  out[3 * i] = E.x;
  out[3 * i + 1] = E.y;
  out[3 * i + 2] = E.z;
}

// ---- launches

static inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_set_params(const FrameParams& p, FrameScratch fs, hipStream_t s) {
  irf_launch(k_set_params, dim3(1), dim3(64), 0, s, p, fs.params);
}

const void* set_params_kernel() { return (const void*)k_set_params; }

void launch_directions(const VolumeSet& vs, FrameScratch fs, hipStream_t s) {
  int maxr = 0;
  for (int v = 0; v < vs.n; v++) maxr = vs.v[v].rays > maxr ? vs.v[v].rays : maxr;
  irf_launch(k_directions, dim3(nblocks(maxr, 256), vs.n), dim3(256), 0, s, vs, fs);
}

void launch_state_compact(const VolumeSet& vs, ObjectBoxes boxes, FrameScratch fs, hipStream_t s) {
  CompactArgs A;
  A.block_base[0] = 0;
  for (int v = 0; v < vs.n; v++) A.block_base[v + 1] = A.block_base[v] + (vs.v[v].n_probes + kCompactBlock - 1) / kCompactBlock;
  if (A.block_base[vs.n] == 0) return;
  irf_launch(k_state_count, dim3(A.block_base[vs.n]), dim3(kCompactBlock), 0, s, vs, boxes, A, fs);
  irf_launch(k_state_scatter, dim3(A.block_base[vs.n]), dim3(kCompactBlock), 0, s, vs, A, fs);
}

void launch_blend(const VolumeSet& vs, FrameScratch fs, hipStream_t s) {
  if (fs.max_slots == 0) return;
  irf_launch(k_blend_f32, dim3(fs.max_slots), dim3(kBlendBlock), 0, s, vs, fs);
}

void launch_query(const VolumeSet& vs, const float* pos, const float* nrm, const float* view, int64_t n, float* out,
                  hipStream_t s) {
  if (n == 0) return;
  irf_launch(k_query, dim3(nblocks(n, kQueryBlock)), dim3(kQueryBlock), 0, s, vs, pos, nrm, view, n, out);
}

}  // namespace irf
