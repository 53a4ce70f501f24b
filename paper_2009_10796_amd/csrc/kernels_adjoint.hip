// Adjoint of the query, the blend and the hit shading, with the ray hits and
// shadow decisions of the forward frame held fixed (then the frame is a
// smooth function of emitter radiance and input texels, up to the clamp of
// the Chebyshev variance at zero).
//
//  k_query_backward   dLoss/d(texels) of E(X, n, w_o) for a batch of points
//  k_blend_backward   per probe: folds border gradients into their source
//                     texels, passes alpha * gradient to the input texels
//                     (all of it for probes that were not updated) and the
//                     transposed normalised weights to every ray's radiance
//  k_shade_backward   per ray: radiance gradient to the hit's emitter and,
//                     through albedo, to the previous-frame query at the hit
//
// Gradient atlases have the layout of the atlases (irradiance [P][8][8][4],
// distance [P][16][16][2], float32) and accumulate with atomic adds.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace irf {

template <int M>
__device__ __forceinline__ void scatter_bilinear(float* tile, int nch, int stride, float3 v, const float* g) {
  int x0, y0;
  float fx, fy;
  tile_footprint<M>(v, x0, y0, fx, fy);
  const float bw[4] = {(1.0f - fx) * (1.0f - fy), fx * (1.0f - fy), (1.0f - fx) * fy, fx * fy};
  const int idx[4] = {y0 * M + x0, y0 * M + x0 + 1, (y0 + 1) * M + x0, (y0 + 1) * M + x0 + 1};
  for (int t = 0; t < 4; t++)
    for (int c = 0; c < nch; c++) atomicAdd(&tile[idx[t] * stride + c], bw[t] * g[c]);
}

// Reverse pass of one volume's cage query (forward: volume_query).
__device__ inline void volume_query_backward(const VolumeGPU& V, float3 X, float3 n, float3 wo, float3 g, float* gI,
                                             float* gD) {
  float u[3] = {(X.x - V.origin[0]) * V.inv_spacing[0], (X.y - V.origin[1]) * V.inv_spacing[1],
                (X.z - V.origin[2]) * V.inv_spacing[2]};
  int gi[3];
  float f[3];
  for (int a = 0; a < 3; a++) {
    gi[a] = (int)clampf(floorf(u[a]), 0.0f, (float)(V.counts[a] - 2));
    f[a] = clampf(u[a] - (float)gi[a], 0.0f, 1.0f);
  }
  float D = fminf(V.spacing[0], fminf(V.spacing[1], V.spacing[2]));
  float sb = 0.75f * D * V.bias;
  float3 Xb = f3(fmaf(fmaf(0.2f, n.x, 0.8f * wo.x), sb, X.x), fmaf(fmaf(0.2f, n.y, 0.8f * wo.y), sb, X.y),
                 fmaf(fmaf(0.2f, n.z, 0.8f * wo.z), sb, X.z));
  // first pass: weights and the normalised result
  float w[8], wtb[8], r8[8];
  float3 e[8], zd[8];
  float2 mm[8];
  int qs[8];
  bool cheb[8];
  int used = 0;
  float W = 0.0f;
  float3 E = f3(0.0f, 0.0f, 0.0f);
  for (int c = 0; c < 8; c++) {
    int cb0 = c & 1, cb1 = (c >> 1) & 1, cb2 = (c >> 2) & 1;
    int q = storage_index(V, gi[0] + cb0, gi[1] + cb1, gi[2] + cb2);
    if (!sampled_state(V.states[q])) continue;
    float wt = (cb0 ? f[0] : 1.0f - f[0]) * (cb1 ? f[1] : 1.0f - f[1]) * (cb2 ? f[2] : 1.0f - f[2]);
    float3 P = probe_position(V, q);
    float3 toP = normalize_or_zero(P - X);
    float h = (1.0f + dot(n, toP)) * 0.5f;
    float ww = wt * fmaf(h, h, 0.2f);
    wtb[used] = ww;
    float3 z = Xb - P;
    float r = length(z);
    cheb[used] = false;
    if (r > 0.0f) {
      zd[used] = (1.0f / r) * z;
      mm[used] = sample_distance(V, q, zd[used]);
      if (r > mm[used].x) {
        float var = fmaxf(fmaf(-mm[used].x, mm[used].x, mm[used].y), 0.0f);
        float dl = r - mm[used].x;
        float ch = var / fmaf(dl, dl, var);
        float p = ch;
        for (int k = 1; k < V.cheb_power; k++) p *= ch;
        ww *= p;
        cheb[used] = true;
      }
    }
    r8[used] = r;
    qs[used] = q;
    w[used] = ww;
    e[used] = sample_irradiance(V, q, n);
    E = E + ww * e[used];
    W += ww;
    used++;
  }
  if (!(W > 0.0f)) return;
  const float iW = 1.0f / W;
  E = iW * E;
  for (int i = 0; i < used; i++) {
    const float ge[3] = {g.x * w[i] * iW, g.y * w[i] * iW, g.z * w[i] * iW};
    scatter_bilinear<kIrrTile>(gI + (size_t)qs[i] * kIrrTexels * 4, 3, 4, n, ge);
    if (!cheb[i]) continue;
    const float gw = (g.x * (e[i].x - E.x) + g.y * (e[i].y - E.y) + g.z * (e[i].z - E.z)) * iW;
    const float mu = mm[i].x, mu2 = mm[i].y;
    const float raw = fmaf(-mu, mu, mu2);
    const float var = fmaxf(raw, 0.0f);
    const float dl = r8[i] - mu;
    const float den = fmaf(dl, dl, var);
    const float ch = var / den;
    const float dch_dvar = dl * dl / (den * den);
    const float dch_ddl = -2.0f * dl * var / (den * den);
    const float dvar_dmu = raw > 0.0f ? -2.0f * mu : 0.0f, dvar_dmu2 = raw > 0.0f ? 1.0f : 0.0f;
    float dwv = (float)V.cheb_power;
    for (int k = 1; k < V.cheb_power; k++) dwv *= ch;
    const float gwv = gw * wtb[i] * dwv;
    const float gd[2] = {gwv * (dch_dvar * dvar_dmu - dch_ddl), gwv * dch_dvar * dvar_dmu2};
    scatter_bilinear<kDistTile>(gD + (size_t)qs[i] * kDistTexels * 2, 2, 2, zd[i], gd);
  }
}

__device__ inline void query_backward(const VolumeSet& vs, const GradSet& G, float3 X, float3 n, float3 wo, float3 g) {
  float Wt = 0.0f;
  for (int v = 0; v < vs.n; v++) {
    if (Wt >= 1.0f) break;
    const VolumeGPU& V = vs.v[v];
    float wv = volume_weight(V, X);
    float wuse = (v == vs.n - 1) ? 1.0f - Wt : fminf(wv, 1.0f - Wt);
    if (wuse > 0.0f) {
      volume_query_backward(V, X, n, wo, wuse * g, G.irr[v], G.dist[v]);
      Wt += wuse;
    }
  }
}

__global__ void k_query_backward(VolumeSet vs, const float* pos, const float* nrm, const float* view, int64_t n,
                                 const float* gout, GradSet G) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float3 X = f3(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
    float3 N = f3(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]);
    float3 Wo = f3(view[3 * i], view[3 * i + 1], view[3 * i + 2]);
    query_backward(vs, G, X, N, Wo, f3(gout[3 * i], gout[3 * i + 1], gout[3 * i + 2]));
  }
}

__device__ __forceinline__ bool was_active(uint8_t s) {
  return s == IRF_NEWLY_AWAKE || s == IRF_NEWLY_VIGILANT || s == IRF_AWAKE || s == IRF_VIGILANT;
}

// Sum of the output gradients of interior cell (x, y) and of the border cells
// that repeat it (the border is a copy of the interior).
template <int M>
__device__ __forceinline__ float folded(const float* g, int stride, int c, int x, int y) {
  constexpr int k = M - 2;
  auto at = [&](int xx, int yy) { return g[(yy * M + xx) * stride + c]; };
  float s = at(x, y);
  if (y == 1) s += at(k + 1 - x, 0);
  if (y == k) s += at(k + 1 - x, k + 1);
  if (x == 1) s += at(0, k + 1 - y);
  if (x == k) s += at(k + 1, k + 1 - y);
  if (x == k && y == k) s += at(0, 0);
  if (x == 1 && y == k) s += at(k + 1, 0);
  if (x == k && y == 1) s += at(0, k + 1);
  if (x == 1 && y == 1) s += at(k + 1, k + 1);
  return s;
}

constexpr int kBwdBlock = 256;

// One workgroup per probe of every volume.  prev: the frame's input atlases
// and the states after its state step.
__global__ __launch_bounds__(kBwdBlock) void k_blend_backward(VolumeSet prev, FrameScratch fs, GradSet Gnew,
                                                              GradSet Gprev) {
  __shared__ float s_g[36][3];
  __shared__ float s_iW[36];
  const FrameCounters& C = *fs.counters;
  int gq = blockIdx.x;
  int v = 0;
  while (v + 1 < prev.n && gq >= prev.v[v + 1].probe_base) v++;
  const VolumeGPU& V = prev.v[v];
  const int q = gq - V.probe_base;
  if (q >= V.n_probes) return;
  const float* gi = Gnew.irr[v] + (size_t)q * kIrrTexels * 4;
  const float* gd = Gnew.dist[v] + (size_t)q * kDistTexels * 2;
  float* pi = Gprev.irr[v] + (size_t)q * kIrrTexels * 4;
  float* pd = Gprev.dist[v] + (size_t)q * kDistTexels * 2;
  const uint8_t st = V.states[q];
  if (!was_active(st)) {
    // not updated: the output texels are the input texels
    for (int i = threadIdx.x; i < kIrrTexels * 4; i += kBwdBlock) pi[i] += gi[i];
    for (int i = threadIdx.x; i < kDistTexels * 2; i += kBwdBlock) pd[i] += gd[i];
    return;
  }
  const bool fresh = st == IRF_NEWLY_AWAKE || st == IRF_NEWLY_VIGILANT;
  const float ai = fresh ? 0.0f : V.alpha_irr, ad = fresh ? 0.0f : V.alpha_dist;
  const int N = V.rays;
  const float4* om = fs.omega + V.omega_base;
  const int t = threadIdx.x;
  if (t < 36) {
    const int x = t % 6 + 1, y = t / 6 + 1;
    float3 nt = texel_direction<kIrrTile>(x, y);
    float W = 0.0f;
    for (int r = 0; r < N; r++) {
      float4 o = om[r];
      W += fmaxf(0.0f, fmaf(nt.x, o.x, fmaf(nt.y, o.y, nt.z * o.z)));
    }
    s_iW[t] = W > 0.0f ? 1.0f / W : 0.0f;
    for (int c = 0; c < 3; c++) {
      float g = folded<kIrrTile>(gi, 4, c, x, y);
      s_g[t][c] = g;
      pi[(y * kIrrTile + x) * 4 + c] += (W > 0.0f ? ai : 1.0f) * g;
    }
  }
  if (t < 196) {
    const int x = t % 14 + 1, y = t / 14 + 1;
    float3 nt = texel_direction<kDistTile>(x, y);
    // a zero weight sum keeps the texel (same float32 weights as the forward)
    float W = 0.0f;
    for (int r = 0; r < N; r++) {
      float4 o = om[r];
      float c = fmaf(nt.x, o.x, fmaf(nt.y, o.y, nt.z * o.z));
      if (c > 0.0f) W += pow_weight(c, V);
    }
    const bool any = W > 0.0f;
    for (int c = 0; c < 2; c++) pd[(y * kDistTile + x) * 2 + c] += (any ? ad : 1.0f) * folded<kDistTile>(gd, 2, c, x, y);
  }
  __syncthreads();
  // the probe's slot in the frame (active lists are ascending per volume)
  int lo = C.slot_base[v], hi = C.slot_base[v + 1] - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (fs.active[mid] < gq) lo = mid + 1;
    else hi = mid;
  }
  const int64_t base = C.ray_base[v] + (int64_t)(lo - C.slot_base[v]) * N;
  for (int r = t; r < N; r += kBwdBlock) {
    float4 o = om[r];
    float3 acc = f3(0.0f, 0.0f, 0.0f);
    for (int k = 0; k < 36; k++) {
      float3 nt = texel_direction<kIrrTile>(k % 6 + 1, k / 6 + 1);
      float w = fmaxf(0.0f, fmaf(nt.x, o.x, fmaf(nt.y, o.y, nt.z * o.z))) * s_iW[k];
      acc = acc + w * f3(s_g[k][0], s_g[k][1], s_g[k][2]);
    }
    fs.grad_rays[base + r] = make_float4((1.0f - ai) * acc.x, (1.0f - ai) * acc.y, (1.0f - ai) * acc.z, 0.0f);
  }
}

__device__ __forceinline__ int64_t ray_volume(const VolumeSet& vs, const FrameCounters& C, int64_t id) {
  int v = 0;
  while (v + 1 < vs.n && id >= C.ray_base[v + 1]) v++;
  return v;
}

// Per ray of the frame: emitter gradient and the previous-frame query at the
// hit (front faces only; misses and backfaces carry constants).
__global__ void k_shade_backward(VolumeSet prev, SceneGPU sc, FrameScratch fs, GradSet Gprev, float* g_emission) {
  const FrameCounters& C = *fs.counters;
  const int64_t total = C.ray_base[prev.n];
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
       id += (int64_t)gridDim.x * blockDim.x) {
    HitRec h = fs.hits[id];
    if (h.tri < 0) continue;
    const int v = (int)ray_volume(prev, C, id);
    const VolumeGPU& V = prev.v[v];
    const int64_t local = id - C.ray_base[v];
    const int slot = (int)(local / V.rays), r = (int)(local - (int64_t)slot * V.rays);
    const int q = fs.active[C.slot_base[v] + slot] - V.probe_base;
    float4 w4 = fs.omega[V.omega_base + r];
    float3 w = f3(w4.x, w4.y, w4.z);
    const float4* tp = sc.tris + (size_t)h.tri * 3;
    float4 a = tp[0], b = tp[1], c = tp[2];
    float3 ng = normalize_or_zero(cross(f3(b.x - a.x, b.y - a.y, b.z - a.z), f3(c.x - a.x, c.y - a.y, c.z - a.z)));
    if (dot(w, ng) > 0.0f) continue;
    float4 g = fs.grad_rays[id];
    const int m = __float_as_int(c.w);
    atomicAdd(&g_emission[3 * m + 0], g.x);
    atomicAdd(&g_emission[3 * m + 1], g.y);
    atomicAdd(&g_emission[3 * m + 2], g.z);
    float4 al = sc.albedo[m];
    float3 o = probe_position(V, q);
    float3 X = f3(fmaf(h.t, w.x, o.x), fmaf(h.t, w.y, o.y), fmaf(h.t, w.z, o.z));
    query_backward(prev, Gprev, X, ng, f3(-w.x, -w.y, -w.z), f3(al.x * g.x, al.y * g.y, al.z * g.z));
  }
}

__global__ void k_set_emission(const float* src, float4* dst, int m) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) dst[i] = make_float4(src[3 * i], src[3 * i + 1], src[3 * i + 2], 0.0f);
}

__global__ void k_copy_words(uint32_t* dst, const uint32_t* src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void k_copy_bytes(uint8_t* dst, const uint8_t* src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

void launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return;
  if (bytes % 4 == 0 && ((uintptr_t)dst & 3) == 0 && ((uintptr_t)src & 3) == 0)
    irf_launch(k_copy_words, dim3(1024), dim3(256), 0, s, (uint32_t*)dst, (const uint32_t*)src, bytes / 4);
  else
    irf_launch(k_copy_bytes, dim3(1024), dim3(256), 0, s, (uint8_t*)dst, (const uint8_t*)src, bytes);
}

void launch_set_emission(const float* src, float4* dst, int m, hipStream_t s) {
  irf_launch(k_set_emission, dim3((m + 255) / 256), dim3(256), 0, s, src, dst, m);
}

void launch_query_backward(const VolumeSet& vs, const float* pos, const float* nrm, const float* view, int64_t n,
                           const float* gout, const GradSet& G, hipStream_t s) {
  if (n == 0) return;
  int64_t blocks = (n + 255) / 256;
  irf_launch(k_query_backward, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, vs, pos, nrm,
                     view, n, gout, G);
}

void launch_update_backward(const VolumeSet& prev, SceneGPU sc, FrameScratch fs, const GradSet& Gnew,
                            const GradSet& Gprev, float* g_emission, hipStream_t s) {
  int P = 0;
  for (int v = 0; v < prev.n; v++) P += prev.v[v].n_probes;
  if (P == 0) return;
  irf_launch(k_blend_backward, dim3(P), dim3(kBwdBlock), 0, s, prev, fs, Gnew, Gprev);
  if (fs.max_rays > 0) {
    int64_t blocks = (fs.max_rays + 255) / 256;
    irf_launch(k_shade_backward, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, s, prev, sc,
                       fs, Gprev, g_emission);
  }
}

}  // namespace irf
