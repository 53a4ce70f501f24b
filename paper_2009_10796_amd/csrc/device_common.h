// Device helpers shared by the irf kernels: octahedral map, probe positions,
// tile sampling and the probe query E(X, n, w_o).
#pragma once
#include <hip/hip_runtime.h>

#include "irf_internal.h"

namespace irf {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator*(float s, float3 a) { return f3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ float3 cross(float3 a, float3 b) {
  return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float length(float3 a) { return sqrtf(dot(a, a)); }
__device__ __forceinline__ float3 normalize_or_zero(float3 a) {
  float l = length(a);
  return l > 0.0f ? (1.0f / l) * a : f3(0.0f, 0.0f, 0.0f);
}
__device__ __forceinline__ float signnz(float x) { return x >= 0.0f ? 1.0f : -1.0f; }
__device__ __forceinline__ float clampf(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }
// Hardware reciprocal and reciprocal square root (1 ulp), for the query's
// inner loop.
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq_fast(float x) { return __builtin_amdgcn_rsqf(x); }

// Octahedral map of the unit sphere onto [-1,1]^2 (Cigolle et al. 2014).
__device__ __forceinline__ float2 oct_encode(float3 v) {
  float l1 = fabsf(v.x) + fabsf(v.y) + fabsf(v.z);
  float x = v.x / l1, y = v.y / l1;
  if (v.z < 0.0f) {
    float nx = (1.0f - fabsf(y)) * signnz(x);
    float ny = (1.0f - fabsf(x)) * signnz(y);
    x = nx;
    y = ny;
  }
  return make_float2(x, y);
}

__device__ __forceinline__ float3 oct_decode(float x, float y) {
  float z = 1.0f - fabsf(x) - fabsf(y);
  if (z < 0.0f) {
    float nx = (1.0f - fabsf(y)) * signnz(x);
    float ny = (1.0f - fabsf(x)) * signnz(y);
    x = nx;
    y = ny;
  }
  return normalize_or_zero(f3(x, y, z));
}

// Direction of interior cell (x, y), 1 <= x, y <= M-2, of an M x M tile.
template <int M>
__device__ __forceinline__ float3 texel_direction(int x, int y) {
  constexpr float k = (float)(M - 2);
  return oct_decode((2.0f * (float)(x - 1) + 1.0f) / k - 1.0f, (2.0f * (float)(y - 1) + 1.0f) / k - 1.0f);
}

// Source cell of border cell (x, y): the neighbour across the octahedral
// seam (edges mirror, corners take the opposite interior corner).
template <int M>
__device__ __forceinline__ void border_source(int x, int y, int& sx, int& sy) {
  constexpr int k = M - 2;
  bool bx = (x == 0 || x == k + 1), by = (y == 0 || y == k + 1);
  if (bx && by) {
    sx = (x == 0) ? k : 1;
    sy = (y == 0) ? k : 1;
  } else if (by) {
    sx = k + 1 - x;
    sy = (y == 0) ? 1 : k;
  } else if (bx) {
    sx = (x == 0) ? 1 : k;
    sy = k + 1 - y;
  } else {
    sx = x;
    sy = y;
  }
}

// Bilinear footprint of direction v in an M x M tile.
template <int M>
__device__ __forceinline__ void tile_footprint(float3 v, int& x0, int& y0, float& fx, float& fy) {
  constexpr int k = M - 2;
  float2 p = oct_encode(v);
  float cx = fmaf(fmaf(0.5f, p.x, 0.5f), (float)k, 0.5f);
  float cy = fmaf(fmaf(0.5f, p.y, 0.5f), (float)k, 0.5f);
  x0 = min(max((int)floorf(cx), 0), k);
  y0 = min(max((int)floorf(cy), 0), k);
  fx = clampf(cx - (float)x0, 0.0f, 1.0f);
  fy = clampf(cy - (float)y0, 0.0f, 1.0f);
}

// The same footprint with the octahedral projection's division done by the
// hardware reciprocal (query path).
template <int M>
__device__ __forceinline__ void tile_footprint_fast(float3 v, int& x0, int& y0, float& fx, float& fy) {
  constexpr int k = M - 2;
  const float il1 = rcp_fast(fabsf(v.x) + fabsf(v.y) + fabsf(v.z));
  float x = v.x * il1, y = v.y * il1;
  if (v.z < 0.0f) {
    const float nx = (1.0f - fabsf(y)) * signnz(x);
    const float ny = (1.0f - fabsf(x)) * signnz(y);
    x = nx;
    y = ny;
  }
  const float cx = fmaf(fmaf(0.5f, x, 0.5f), (float)k, 0.5f);
  const float cy = fmaf(fmaf(0.5f, y, 0.5f), (float)k, 0.5f);
  x0 = min(max((int)floorf(cx), 0), k);
  y0 = min(max((int)floorf(cy), 0), k);
  fx = clampf(cx - (float)x0, 0.0f, 1.0f);
  fy = clampf(cy - (float)y0, 0.0f, 1.0f);
}

// Rows of the matrix-core blend's weight matrix: the 36 irradiance interior
// texels padded to 48, then the 196 distance interior texels padded to 208.
constexpr int kRows = 256;
constexpr int kIrrRows = 48;

// Direction i of an n-ray spherical-Fibonacci pattern (Section "Probe
// Update": the same rotated pattern for every probe of the frame), rotated by
// the row-major matrix R.
__device__ __forceinline__ float3 sf_direction(int i, int n, const float* R) {
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

// Distance-blend weight cos^p of a positive cosine (square-and-multiply for
// an integer exponent, so every kernel gets the same float32 value).
__device__ __forceinline__ float pow_weight(float c, const VolumeGPU& V) {
  if (V.cos_power_int > 0) {
    float r = 1.0f, b = c;
    int e = V.cos_power_int;
    while (e) {
      if (e & 1) r *= b;
      b *= b;
      e >>= 1;
    }
    return r;
  }
  return powf(c, V.cos_power);
}

// Section "Tracking Windows": a tracking volume is a circular buffer, the
// storage slot of logical grid index i along an axis being (i + phase) mod n
// (phase 0 for other volumes).  Both arguments below are within one period.
__device__ __forceinline__ int slot_of(int i, int phase, int n) {
  int x = i + phase;
  return x >= n ? x - n : x;
}
__device__ __forceinline__ int logical_of(int s, int phase, int n) {
  int x = s - phase;
  return x < 0 ? x + n : x;
}

// Probe index x + nx (y + ny z) of the storage slots: every partial product
// is below the volume's probe count (at most 2^22), so 24-bit multiplies
// (full rate) are exact.
__device__ __forceinline__ int storage_index(const VolumeGPU& V, int i, int j, int k) {
  const uint32_t yz = (uint32_t)slot_of(j, V.phase[1], V.counts[1]) +
                      __umul24((uint32_t)V.counts[1], (uint32_t)slot_of(k, V.phase[2], V.counts[2]));
  return (int)((uint32_t)slot_of(i, V.phase[0], V.counts[0]) + __umul24((uint32_t)V.counts[0], yz));
}

__device__ __forceinline__ void logical_index(const VolumeGPU& V, int q, int g[3]) {
  g[0] = logical_of(q % V.counts[0], V.phase[0], V.counts[0]);
  g[1] = logical_of((q / V.counts[0]) % V.counts[1], V.phase[1], V.counts[1]);
  g[2] = logical_of(q / (V.counts[0] * V.counts[1]), V.phase[2], V.counts[2]);
}

__device__ __forceinline__ float3 probe_position(const VolumeGPU& V, int q) {
  int g[3];
  logical_index(V, q, g);
  int i = g[0], j = g[1], k = g[2];
  float3 P = f3(fmaf((float)i, V.spacing[0], V.origin[0]), fmaf((float)j, V.spacing[1], V.origin[1]),
                fmaf((float)k, V.spacing[2], V.origin[2]));
  if (V.offsets) {
    P.x += V.offsets[3 * q + 0];
    P.y += V.offsets[3 * q + 1];
    P.z += V.offsets[3 * q + 2];
  }
  return P;
}

__device__ __forceinline__ float3 load_irr(const VolumeGPU& V, int idx) {
  if (V.atlas_f16) {
    h4 h = ((const h4*)V.irr)[idx];
    return f3((float)h.x, (float)h.y, (float)h.z);
  }
  float4 f = ((const float4*)V.irr)[idx];
  return f3(f.x, f.y, f.z);
}

__device__ __forceinline__ float2 load_dist(const VolumeGPU& V, int idx) {
  if (V.atlas_f16) {
    h2 h = ((const h2*)V.dist)[idx];
    return make_float2((float)h.x, (float)h.y);
  }
  return ((const float2*)V.dist)[idx];
}

__device__ __forceinline__ float3 sample_irradiance(const VolumeGPU& V, int q, float3 n) {
  int x0, y0;
  float fx, fy;
  tile_footprint<kIrrTile>(n, x0, y0, fx, fy);
  int b = q * kIrrTexels + y0 * kIrrTile + x0;
  float3 a = load_irr(V, b), c = load_irr(V, b + 1);
  float3 d = load_irr(V, b + kIrrTile), e = load_irr(V, b + kIrrTile + 1);
  float3 top = (1.0f - fx) * a + fx * c;
  float3 bot = (1.0f - fx) * d + fx * e;
  return (1.0f - fy) * top + fy * bot;
}

__device__ __forceinline__ float2 sample_distance(const VolumeGPU& V, int q, float3 v) {
  int x0, y0;
  float fx, fy;
  tile_footprint<kDistTile>(v, x0, y0, fx, fy);
  int b = q * kDistTexels + y0 * kDistTile + x0;
  float2 a = load_dist(V, b), c = load_dist(V, b + 1);
  float2 d = load_dist(V, b + kDistTile), e = load_dist(V, b + kDistTile + 1);
  float tx = (1.0f - fx) * a.x + fx * c.x, ty = (1.0f - fx) * a.y + fx * c.y;
  float bx = (1.0f - fx) * d.x + fx * e.x, by = (1.0f - fx) * d.y + fx * e.y;
  return make_float2((1.0f - fy) * tx + fy * bx, (1.0f - fy) * ty + fy * by);
}

__device__ __forceinline__ bool sampled_state(uint8_t s) { return s == IRF_AWAKE || s == IRF_VIGILANT; }

// Section "Perception-based exponential encoding": irradiance texels store the
// new mean to the power 1/gamma (and blend in that encoding); the query
// raises each probe's sample to gamma/2, blends on that curve and squares.
__device__ __forceinline__ float encode_irr(const VolumeGPU& V, float x) {
  return V.gamma == 1.0f ? x : powf(fmaxf(x, 0.0f), V.inv_gamma);
}

__device__ __forceinline__ float3 decode_irr_half(const VolumeGPU& V, float3 e) {
  return f3(powf(fmaxf(e.x, 0.0f), V.half_gamma), powf(fmaxf(e.y, 0.0f), V.half_gamma),
            powf(fmaxf(e.z, 0.0f), V.half_gamma));
}

// Section "Fast Convergence Heuristics": the irradiance hysteresis of one
// texel from the largest per-channel change in stored units between the new
// (encoded) value and the stored one -- lowered by 0.15 (not below 0) above
// 0.25, and 0 above 0.8.
__device__ __forceinline__ float texel_alpha(const VolumeGPU& V, float alpha, float3 enc, float3 old) {
  if (!V.thresholds) return alpha;
  float change = fmaxf(fabsf(enc.x - old.x), fmaxf(fabsf(enc.y - old.y), fabsf(enc.z - old.z)));
  float a = alpha;
  if (change > 0.25f) a = fmaxf(0.0f, a - 0.15f);
  if (change > 0.8f) a = 0.0f;
  return a;
}

// The new stored irradiance texel (Eq. U in the stored encoding) from the
// stored one and the new normalised mean.  The blend is written as one
// fused multiply-add over a rounded product, so that every kernel (and every
// tile shape) that inlines it rounds the same way.
__device__ __forceinline__ float3 irr_texel_update(const VolumeGPU& V, float alpha, float3 old, float3 mean) {
  float3 e = f3(encode_irr(V, mean.x), encode_irr(V, mean.y), encode_irr(V, mean.z));
  float a = texel_alpha(V, alpha, e, old);
  const float b = 1.0f - a;
  return f3(fmaf(a, old.x, b * e.x), fmaf(a, old.y, b * e.y), fmaf(a, old.z, b * e.z));
}

template <bool F16>
__device__ __forceinline__ float3 load_irr_t(const VolumeGPU& V, int idx) {
  if constexpr (F16) {
    const h4 h = ((const h4*)V.irr)[idx];
    return f3((float)h.x, (float)h.y, (float)h.z);
  } else {
    const float4 f = ((const float4*)V.irr)[idx];
    return f3(f.x, f.y, f.z);
  }
}

template <bool F16>
__device__ __forceinline__ float2 load_dist_t(const VolumeGPU& V, int idx) {
  if constexpr (F16) {
    const h2 h = ((const h2*)V.dist)[idx];
    return make_float2((float)h.x, (float)h.y);
  } else {
    return ((const float2*)V.dist)[idx];
  }
}

// Two horizontally adjacent texels of one tile row (x, x + 1; contiguous in
// the atlas, the second never past the row) with one wide load: 16 bytes for
// a float2 distance pair or a half4 irradiance pair, 8 for a half2 distance
// pair.  Atlas rows start at the texel size's alignment, so the wide load is
// aligned to the texel, not to its own width (dword alignment is what global
// loads need).
typedef float f4_a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef _Float16 h8_a8 __attribute__((ext_vector_type(8), aligned(8)));
typedef _Float16 h4_a4 __attribute__((ext_vector_type(4), aligned(4)));

template <bool F16>
__device__ __forceinline__ void load_irr_pair_t(const VolumeGPU& V, int idx, float3& a, float3& b) {
  if constexpr (F16) {
    const h8_a8 h = *(const h8_a8*)((const h4*)V.irr + idx);
    a = f3((float)h[0], (float)h[1], (float)h[2]);
    b = f3((float)h[4], (float)h[5], (float)h[6]);
  } else {
    a = load_irr_t<false>(V, idx);
    b = load_irr_t<false>(V, idx + 1);
  }
}

template <bool F16>
__device__ __forceinline__ void load_dist_pair_t(const VolumeGPU& V, int idx, float2& a, float2& b) {
  if constexpr (F16) {
    const h4_a4 h = *(const h4_a4*)((const h2*)V.dist + idx);
    a = make_float2((float)h[0], (float)h[1]);
    b = make_float2((float)h[2], (float)h[3]);
  } else {
    const f4_a8 f = *(const f4_a8*)((const float2*)V.dist + idx);
    a = make_float2(f[0], f[1]);
    b = make_float2(f[2], f[3]);
  }
}

// One volume's 8-probe cage (Section "Probe Query"): trilinear x backface x
// Chebyshev visibility at the point moved by the self-shadow bias (Eq. 1);
// normalised.  Returns zero when no probe carries weight.
// `look`: the direction the irradiance texels are sampled in (the normal for
// the irradiance query; the second-order glossy pass samples the probes'
// filtered radiance in a mirror direction).
// The cage is unrolled: the eight state bytes are fetched together, and each
// probe's texel fetches carry no format branch between them (F16: half
// atlases), so they are in flight together.
template <bool F16>
__device__ __forceinline__ float3 volume_query_t(const VolumeGPU& V, float3 X, float3 n, float3 wo, float3 look) {
  const float Xa[3] = {X.x, X.y, X.z};
  int g[3];
  float f[3], Pa[3][2];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const float u = (Xa[a] - V.origin[a]) * V.inv_spacing[a];
    const float fl = floorf(u);
    g[a] = (int)clampf(fl, 0.0f, (float)(V.counts[a] - 2));
    f[a] = clampf(u - (float)g[a], 0.0f, 1.0f);
    // probe coordinates of the cage's two planes along the axis, from the
    // logical index (as probe_position computes them)
    Pa[a][0] = fmaf((float)g[a], V.spacing[a], V.origin[a]);
    Pa[a][1] = fmaf((float)(g[a] + 1), V.spacing[a], V.origin[a]);
  }
  const float D = fminf(V.spacing[0], fminf(V.spacing[1], V.spacing[2]));
  const float sb = 0.75f * D * V.bias;
  const float3 Xb = f3(fmaf(fmaf(0.2f, n.x, 0.8f * wo.x), sb, X.x), fmaf(fmaf(0.2f, n.y, 0.8f * wo.y), sb, X.y),
                       fmaf(fmaf(0.2f, n.z, 0.8f * wo.z), sb, X.z));
  // the irradiance lookup direction is the same for every probe of the cage
  int ix, iy;
  float ifx, ify;
  tile_footprint_fast<kIrrTile>(look, ix, iy, ifx, ify);
  const int irr_off = iy * kIrrTile + ix;
  // the cage's storage slots, two per axis, and its eight probe indices
  int sx[2], sy[2], sz[2];
#pragma unroll
  for (int b = 0; b < 2; b++) {
    sx[b] = slot_of(g[0] + b, V.phase[0], V.counts[0]);
    sy[b] = slot_of(g[1] + b, V.phase[1], V.counts[1]);
    sz[b] = slot_of(g[2] + b, V.phase[2], V.counts[2]);
  }
  int q[8];
  bool use[8];
#pragma unroll
  for (int c = 0; c < 8; c++) {
    const uint32_t yz = (uint32_t)sy[(c >> 1) & 1] + __umul24((uint32_t)V.counts[1], (uint32_t)sz[c >> 2]);
    q[c] = (int)((uint32_t)sx[c & 1] + __umul24((uint32_t)V.counts[0], yz));
  }
#pragma unroll
  for (int c = 0; c < 8; c++) use[c] = sampled_state(V.states[q[c]]);
  float3 acc = f3(0.0f, 0.0f, 0.0f);
  float W = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; c++) {
    if (!use[c]) continue;
    const int cb0 = c & 1, cb1 = (c >> 1) & 1, cb2 = (c >> 2) & 1;
    const float wt = (cb0 ? f[0] : 1.0f - f[0]) * (cb1 ? f[1] : 1.0f - f[1]) * (cb2 ? f[2] : 1.0f - f[2]);
    float3 P = f3(Pa[0][cb0], Pa[1][cb1], Pa[2][cb2]);
    if (V.offsets) {
      P.x += V.offsets[3 * q[c] + 0];
      P.y += V.offsets[3 * q[c] + 1];
      P.z += V.offsets[3 * q[c] + 2];
    }
    // the probe's irradiance texels do not depend on its weight: fetch first
    const int bi = q[c] * kIrrTexels + irr_off;
    float3 ea, ec, ed, ee;
    load_irr_pair_t<F16>(V, bi, ea, ec);
    load_irr_pair_t<F16>(V, bi + kIrrTile, ed, ee);
    const float3 toP = P - X;
    const float d2 = dot(toP, toP);
    const float h = fmaf(d2 > 0.0f ? dot(n, toP) * rsq_fast(d2) : 0.0f, 0.5f, 0.5f);
    float w = wt * fmaf(h, h, 0.2f);
    const float3 z = Xb - P;
    const float r2 = dot(z, z);
    if (r2 > 0.0f) {
      const float r = r2 * rsq_fast(r2);
      int x0, y0;
      float fx, fy;
      tile_footprint_fast<kDistTile>(z, x0, y0, fx, fy);   // the octahedral map is scale-free
      const int b = q[c] * kDistTexels + y0 * kDistTile + x0;
      float2 da, dc, dd, de;
      load_dist_pair_t<F16>(V, b, da, dc);
      load_dist_pair_t<F16>(V, b + kDistTile, dd, de);
      const float mx = (1.0f - fy) * ((1.0f - fx) * da.x + fx * dc.x) + fy * ((1.0f - fx) * dd.x + fx * de.x);
      if (r > mx) {
        const float my = (1.0f - fy) * ((1.0f - fx) * da.y + fx * dc.y) + fy * ((1.0f - fx) * dd.y + fx * de.y);
        const float var = fmaxf(fmaf(-mx, mx, my), 0.0f);
        const float dl = r - mx;
        const float den = fmaf(dl, dl, var);
        const float ch = den > 0.0f ? var * rcp_fast(den) : 0.0f;
        float p = ch;
        for (int e = 1; e < V.cheb_power; e++) p *= ch;
        w *= p;
      }
    }
    float3 e = (1.0f - ify) * ((1.0f - ifx) * ea + ifx * ec) + ify * ((1.0f - ifx) * ed + ifx * ee);
    if (V.gamma != 1.0f) e = decode_irr_half(V, e);
    acc = acc + w * e;
    W += w;
  }
  if (!(W > 0.0f)) return f3(0.0f, 0.0f, 0.0f);
  const float3 r = rcp_fast(W) * acc;
  return V.gamma != 1.0f ? f3(r.x * r.x, r.y * r.y, r.z * r.z) : r;
}

__device__ __forceinline__ float3 volume_query(const VolumeGPU& V, float3 X, float3 n, float3 wo, float3 look) {
  return V.atlas_f16 ? volume_query_t<true>(V, X, n, wo, look) : volume_query_t<false>(V, X, n, wo, look);
}

// Section "Multiple Probe Volumes": a volume's weight falls linearly from 1 to
// 0 over its last grid cell along each axis (product over axes); for a volume
// that tracks the camera the transition region is tightened by one cell and
// centred on the camera.
__device__ __forceinline__ float volume_weight(const VolumeGPU& V, float3 X) {
  float wv = 1.0f;
  const float Xa[3] = {X.x, X.y, X.z};
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (V.tracking) {
      float h = 0.5f * (float)(V.counts[a] - 1) - 1.0f;
      wv *= clampf(h - fabsf(Xa[a] - V.camera[a]) * V.inv_spacing[a], 0.0f, 1.0f);
    } else {
      float u = (Xa[a] - V.origin[a]) * V.inv_spacing[a];
      wv *= clampf(fminf(u, (float)(V.counts[a] - 1) - u), 0.0f, 1.0f);
    }
  }
  return wv;
}

// Cascaded volumes (Section "Multiple Probe Volumes"): densest first, linear
// fall-off over the last cell of each axis (product of axes), accumulate
// until the weights reach one; the sparsest volume takes the remainder.
__device__ __forceinline__ float3 query_look(const VolumeSet& vs, float3 X, float3 n, float3 wo, float3 look) {
  float3 E = f3(0.0f, 0.0f, 0.0f);
  float Wt = 0.0f;
  for (int v = 0; v < vs.n; v++) {
    if (Wt >= 1.0f) break;
    const VolumeGPU& V = vs.v[v];
    float wv = volume_weight(V, X);
    float wuse = (v == vs.n - 1) ? 1.0f - Wt : fminf(wv, 1.0f - Wt);
    if (wuse > 0.0f) {
      E = E + wuse * volume_query(V, X, n, wo, look);
      Wt += wuse;
    }
  }
  return E;
}

__device__ __forceinline__ float3 query_irradiance(const VolumeSet& vs, float3 X, float3 n, float3 wo) {
  return query_look(vs, X, n, wo, n);
}

// Query point i of a batch (position, normal and view direction packed xyz).
__device__ __forceinline__ void query_point(const VolumeSet& vs, const float* __restrict__ pos,
                                            const float* __restrict__ nrm, const float* __restrict__ view, int64_t i,
                                            float* __restrict__ out) {
  const float3 X = f3(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
  const float3 N = f3(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]);
  const float3 Wo = f3(view[3 * i], view[3 * i + 1], view[3 * i + 2]);
  const float3 E = query_irradiance(vs, X, N, Wo);
  out[3 * i] = E.x;
  out[3 * i + 1] = E.y;
  out[3 * i + 2] = E.z;
}

}  // namespace irf
