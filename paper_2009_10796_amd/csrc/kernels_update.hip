// The vector-ALU blend of the probe update, and the query kernel.
//
//  k_blend_f32      Eq. U per texel as a normalised weighted average with
//                   hysteresis; one workgroup per active probe with the
//                   probe's rays in LDS (the paper's coherent compute-shader
//                   update), border texels written by their source texel
//  k_query          E(X, n, w_o) for a batch of points
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace irf {

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
      float2 val = make_float2(fmaf(a, old.x, (1.0f - a) * n1), fmaf(a, old.y, (1.0f - a) * n2));
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
  const int64_t i = (int64_t)blockIdx.x * kQueryBlock + threadIdx.x;
  if (i < n) query_point(vs, pos, nrm, view, i, out);
}

// ---- launches

static inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

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
