// Adjoint of the query, the blend and the hit shading, with the ray hits and
// shadow decisions of the forward frame held fixed (then the frame is a
// smooth function of emitter radiance and input texels, up to the clamp of
// the Chebyshev variance at zero).
//
//  query terms        the reverse pass of one query E(X, n, w_o) as one term
//                     per probe of each cage it read: the gradient of that
//                     probe's irradiance sample and of its (mu, mu2) sample,
//                     with the two bilinear footprints they spread over
//  k_blend_backward   per probe: folds border gradients into their source
//                     texels, passes alpha * gradient to the input texels
//                     (all of it for probes that were not updated) and the
//                     transposed normalised weights to every ray's radiance
//  k_shade_terms      per ray: the query terms of the previous-frame query at
//                     its hit (through albedo) and its emitter record
//
// Gradients are summed without atomics, in a fixed order: the terms and
// emitter records of a batch (points or rays, in index order) are sorted by
// key -- probe, then material -- with a stable radix sort (so a key's terms
// stay in point or ray order); each key's run is cut into pieces of 1,024
// terms, each piece summed by one workgroup in a fixed order, and a run of
// several pieces adds its pieces' sums in piece order.  Results are the same
// bit for bit from run to run.  Gradient atlases have the layout of the
// atlases (irradiance [P][8][8][4], distance [P][16][16][2], float32) and
// accumulate (+=).
#include <hip/hip_runtime.h>

#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "device_common.h"

namespace irf {

// One probe's share of a query's reverse pass: the gradient of its
// irradiance sample (RGB) over the bilinear footprint at (ix, iy) with
// fractions (ifx, ify), and of its (mu, mu2) sample over the footprint at
// (dx, dy), (dfx, dfy).
struct Term {
  float ge[3];
  float gd[2];
  float ifx, ify, dfx, dfy;
  uint32_t fp;   // ix | iy << 8 | dx << 16 | dy << 24
};
static_assert(sizeof(Term) == 40, "ten words");

// ---- the terms in FP64
//
// The reverse pass re-evaluates each query's intermediate values in double
// precision from the frame's float32 inputs (points, normals, texels, probe
// grid, ray directions and hit triangles): the Chebyshev factor and its
// derivatives turn on r - mu and mu2 - mu^2, which cancel, so float32
// intermediates would move the gradient of an ill-conditioned probe far more
// than its value.  The gradient is then that of the exact forward at the
// same float32 inputs, to float32 rounding of each term and of the sums.

struct D3 {
  double x, y, z;
};
__device__ __forceinline__ D3 d3(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ D3 d3f(float3 v) { return {(double)v.x, (double)v.y, (double)v.z}; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator*(double s, D3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dotd(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 crossd(D3 a, D3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ D3 normalized(D3 a) {
  const double l = sqrt(dotd(a, a));
  return l > 0.0 ? (1.0 / l) * a : d3(0.0, 0.0, 0.0);
}

// Bilinear footprint of direction v in an M x M tile (octahedral map, the
// interior k = M - 2 cells, taps at floor(c) and floor(c) + 1).
template <int M>
__device__ __forceinline__ void footprint_d(D3 v, int& x0, int& y0, double& fx, double& fy) {
  constexpr int k = M - 2;
  const double l1 = fabs(v.x) + fabs(v.y) + fabs(v.z);
  double x = v.x / l1, y = v.y / l1;
  if (v.z < 0.0) {
    const double nx = (1.0 - fabs(y)) * (x >= 0.0 ? 1.0 : -1.0);
    const double ny = (1.0 - fabs(x)) * (y >= 0.0 ? 1.0 : -1.0);
    x = nx;
    y = ny;
  }
  const double cx = (0.5 * x + 0.5) * k + 0.5, cy = (0.5 * y + 0.5) * k + 0.5;
  x0 = min(max((int)floor(cx), 0), k);
  y0 = min(max((int)floor(cy), 0), k);
  fx = fmin(fmax(cx - (double)x0, 0.0), 1.0);
  fy = fmin(fmax(cy - (double)y0, 0.0), 1.0);
}

__device__ __forceinline__ D3 irr_texel_d(const VolumeGPU& V, int idx) {
  const float4 t = ((const float4*)V.irr)[idx];
  return d3(t.x, t.y, t.z);
}

__device__ __forceinline__ D3 position_d(const VolumeGPU& V, int q) {
  int g[3];
  logical_index(V, q, g);
  D3 P = d3((double)V.origin[0] + (double)g[0] * (double)V.spacing[0],
            (double)V.origin[1] + (double)g[1] * (double)V.spacing[1],
            (double)V.origin[2] + (double)g[2] * (double)V.spacing[2]);
  if (V.offsets) P = P + d3(V.offsets[3 * q], V.offsets[3 * q + 1], V.offsets[3 * q + 2]);
  return P;
}

// Direction of ray i of an n-ray spherical-Fibonacci pattern under the
// frame's rotation R, in double (frac(i * golden ratio) from the 0.64
// fixed-point golden ratio, exact).
__device__ __forceinline__ D3 sf_direction_d(int i, int n, const float* R) {
  const uint64_t fr = (uint64_t)i * 0x9E3779B97F4A7C15ull;
  const double f = (double)(fr >> 11) * 0x1p-53;
  const double z = 1.0 - (2.0 * i + 1.0) / n;
  const double r = sqrt(fmax(0.0, 1.0 - z * z));
  double sn, cs;
  sincospi(2.0 * f, &sn, &cs);
  const D3 p = d3(r * cs, r * sn, z);
  return d3((double)R[0] * p.x + (double)R[1] * p.y + (double)R[2] * p.z,
            (double)R[3] * p.x + (double)R[4] * p.y + (double)R[5] * p.z,
            (double)R[6] * p.x + (double)R[7] * p.y + (double)R[8] * p.z);
}

// Section "Multiple Probe Volumes" cascade weight of X (non-tracking and
// tracking volumes), in double.
__device__ __forceinline__ double volume_weight_d(const VolumeGPU& V, D3 X) {
  const double Xa[3] = {X.x, X.y, X.z};
  double wv = 1.0;
  for (int a = 0; a < 3; a++) {
    if (V.tracking) {
      const double h = 0.5 * (double)(V.counts[a] - 1) - 1.0;
      wv *= fmin(fmax(h - fabs(Xa[a] - (double)V.camera[a]) / (double)V.spacing[a], 0.0), 1.0);
    } else {
      const double u = (Xa[a] - (double)V.origin[a]) / (double)V.spacing[a];
      wv *= fmin(fmax(fmin(u, (double)(V.counts[a] - 1) - u), 0.0), 1.0);
    }
  }
  return wv;
}

// One corner probe of a cage query: its trilinear x backface weight (wtb),
// full weight (ww, with the Chebyshev factor when r > mu), irradiance sample
// and distance sample.
struct Corner {
  bool ok;      // the probe is sampled
  bool cheb;    // the Chebyshev factor applies
  int q;
  double wtb, ww, r, mu, mu2;
  D3 zd, e;
};

__device__ __forceinline__ Corner corner_eval(const VolumeGPU& V, int c, const int* gi, const double* f, D3 X, D3 Xb,
                                              D3 n, int ix, int iy, double ifx, double ify) {
  Corner k;
  const int cb0 = c & 1, cb1 = (c >> 1) & 1, cb2 = (c >> 2) & 1;
  k.q = storage_index(V, gi[0] + cb0, gi[1] + cb1, gi[2] + cb2);
  k.ok = sampled_state(V.states[k.q]);
  k.cheb = false;
  if (!k.ok) return k;
  const double wt = (cb0 ? f[0] : 1.0 - f[0]) * (cb1 ? f[1] : 1.0 - f[1]) * (cb2 ? f[2] : 1.0 - f[2]);
  const D3 P = position_d(V, k.q);
  const D3 toP = normalized(P - X);
  const double h = (1.0 + dotd(n, toP)) * 0.5;
  k.wtb = wt * (h * h + 0.2);
  k.ww = k.wtb;
  const D3 z = Xb - P;
  k.r = sqrt(dotd(z, z));
  if (k.r > 0.0) {
    k.zd = (1.0 / k.r) * z;
    int x0, y0;
    double fx, fy;
    footprint_d<kDistTile>(k.zd, x0, y0, fx, fy);
    const float2* t = (const float2*)V.dist + (size_t)k.q * kDistTexels + y0 * kDistTile + x0;
    const float2 ta = t[0], tc = t[1], td = t[kDistTile], te = t[kDistTile + 1];
    k.mu = (1.0 - fy) * ((1.0 - fx) * ta.x + fx * tc.x) + fy * ((1.0 - fx) * td.x + fx * te.x);
    k.mu2 = (1.0 - fy) * ((1.0 - fx) * ta.y + fx * tc.y) + fy * ((1.0 - fx) * td.y + fx * te.y);
    if (k.r > k.mu) {
      const double var = fmax(k.mu2 - k.mu * k.mu, 0.0);
      const double dl = k.r - k.mu;
      const double den = var + dl * dl;
      const double ch = den > 0.0 ? var / den : 0.0;
      double p = ch;
      for (int j = 1; j < V.cheb_power; j++) p *= ch;
      k.ww *= p;
      k.cheb = true;
    }
  }
  const int b = k.q * kIrrTexels + iy * kIrrTile + ix;
  const D3 ea = irr_texel_d(V, b), ec = irr_texel_d(V, b + 1);
  const D3 ed = irr_texel_d(V, b + kIrrTile), ee = irr_texel_d(V, b + kIrrTile + 1);
  k.e = (1.0 - ify) * ((1.0 - ifx) * ea + ifx * ec) + ify * ((1.0 - ifx) * ed + ifx * ee);
  return k;
}

// Terms of one volume's cage query (forward: volume_query) with upstream
// gradient g: corner c's term in t[c], key[c] its global probe id (`none`
// for a corner without a sampled probe).  Two passes over the corners (the
// weight sum, then the terms) recompute each corner instead of holding all
// eight in registers.
__device__ inline void volume_query_terms(const VolumeGPU& V, D3 X, D3 n, D3 wo, D3 g, Term* t, uint32_t* key,
                                          uint32_t none) {
  const double Xa[3] = {X.x, X.y, X.z};
  int gi[3];
  double f[3];
  for (int a = 0; a < 3; a++) {
    const double u = (Xa[a] - (double)V.origin[a]) / (double)V.spacing[a];
    gi[a] = (int)fmin(fmax(floor(u), 0.0), (double)(V.counts[a] - 2));
    f[a] = fmin(fmax(u - (double)gi[a], 0.0), 1.0);
  }
  const double D = fmin((double)V.spacing[0], fmin((double)V.spacing[1], (double)V.spacing[2]));
  const double sb = 0.75 * D * (double)V.bias;
  const D3 Xb = X + sb * (0.2 * n + 0.8 * wo);
  int ix, iy;
  double ifx, ify;
  footprint_d<kIrrTile>(n, ix, iy, ifx, ify);
  double W = 0.0;
  D3 E = d3(0.0, 0.0, 0.0);
  for (int c = 0; c < 8; c++) {
    const Corner k = corner_eval(V, c, gi, f, X, Xb, n, ix, iy, ifx, ify);
    if (!k.ok) continue;
    E = E + k.ww * k.e;
    W += k.ww;
  }
  if (!(W > 0.0)) {
    for (int c = 0; c < 8; c++) key[c] = none;
    return;
  }
  const double iW = 1.0 / W;
  E = iW * E;
  for (int c = 0; c < 8; c++) {
    const Corner k = corner_eval(V, c, gi, f, X, Xb, n, ix, iy, ifx, ify);
    if (!k.ok) {
      key[c] = none;
      continue;
    }
    Term T;
    T.ge[0] = (float)(g.x * k.ww * iW);
    T.ge[1] = (float)(g.y * k.ww * iW);
    T.ge[2] = (float)(g.z * k.ww * iW);
    T.gd[0] = T.gd[1] = 0.0f;
    T.ifx = (float)ifx;
    T.ify = (float)ify;
    int dx = 0, dy = 0;
    double dfx = 0.0, dfy = 0.0;
    if (k.cheb) {
      const double gw = dotd(g, k.e - E) * iW;
      const double raw = k.mu2 - k.mu * k.mu;
      const double var = fmax(raw, 0.0);
      const double dl = k.r - k.mu;
      const double den = var + dl * dl;
      const double ch = var / den;
      const double dch_dvar = dl * dl / (den * den);
      const double dch_ddl = -2.0 * dl * var / (den * den);
      const double dvar_dmu = raw > 0.0 ? -2.0 * k.mu : 0.0, dvar_dmu2 = raw > 0.0 ? 1.0 : 0.0;
      double dwv = (double)V.cheb_power;
      for (int j = 1; j < V.cheb_power; j++) dwv *= ch;
      const double gwv = gw * k.wtb * dwv;
      T.gd[0] = (float)(gwv * (dch_dvar * dvar_dmu - dch_ddl));
      T.gd[1] = (float)(gwv * dch_dvar * dvar_dmu2);
      footprint_d<kDistTile>(k.zd, dx, dy, dfx, dfy);
    }
    T.dfx = (float)dfx;
    T.dfy = (float)dfy;
    T.fp = (uint32_t)ix | (uint32_t)iy << 8 | (uint32_t)dx << 16 | (uint32_t)dy << 24;
    t[c] = T;
    key[c] = (uint32_t)(V.probe_base + k.q);
  }
}

// Terms of the query over all volumes (8 slots per volume, in volume order),
// each volume's share of the upstream gradient as its weight in the forward
// cascade blend.
__device__ inline void query_terms(const VolumeSet& vs, D3 X, D3 n, D3 wo, D3 g, Term* t, uint32_t* key,
                                   uint32_t none) {
  double Wt = 0.0;
  for (int v = 0; v < vs.n; v++) {
    const VolumeGPU& V = vs.v[v];
    double wuse = 0.0;
    if (Wt < 1.0) {
      const double wv = volume_weight_d(V, X);
      wuse = (v == vs.n - 1) ? 1.0 - Wt : fmin(wv, 1.0 - Wt);
    }
    if (wuse > 0.0) {
      volume_query_terms(V, X, n, wo, wuse * g, t + 8 * v, key + 8 * v, none);
      Wt += wuse;
    } else {
      for (int i = 0; i < 8; i++) key[8 * v + i] = none;
    }
  }
}

// Query terms of points [i0, i0 + n): point i's at (i - i0) * 8 * vs.n.
__global__ __launch_bounds__(256) void k_query_terms(VolumeSet vs, const float* pos, const float* nrm, const float* view, int64_t i0,
                              int64_t n, const float* gout, Term* terms, uint32_t* keys, uint32_t none) {
  const int per = 8 * vs.n;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + j;
    const D3 X = d3(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]);
    const D3 N = d3(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]);
    const D3 Wo = d3(view[3 * i], view[3 * i + 1], view[3 * i + 2]);
    query_terms(vs, X, N, Wo, d3(gout[3 * i], gout[3 * i + 1], gout[3 * i + 2]), terms + j * per, keys + j * per,
                none);
  }
}

__global__ void k_fill_words(uint32_t* p, uint32_t value, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// Segments of a sorted key array: keys below `none` get [start, end).
__global__ void k_segments(const uint32_t* keys, int64_t n, uint32_t none, uint32_t* start, uint32_t* end) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = keys[i];
    if (k >= none) continue;
    if (i == 0 || keys[i - 1] != k) start[k] = (uint32_t)i;
    if (i == n - 1 || keys[i + 1] != k) end[k] = (uint32_t)(i + 1);
  }
}

// Pieces: each segment (a probe's or a material's terms, in sorted order)
// is cut into pieces of kPieceTerms consecutive terms.  A piece is summed by
// one workgroup in a fixed order; a segment of one piece adds its sum to the
// gradient directly, a longer one stores its pieces' sums and k_finish_pieces
// adds them in piece order.  The cut depends only on the sorted terms, so the
// result is the same from run to run, and no workgroup sums more than
// kPieceTerms terms however the terms crowd onto a few probes.
constexpr int kPieceTerms = 1024;
constexpr int kPieceWaves = 4;
constexpr int kWaveTerms = kPieceTerms / kPieceWaves;
constexpr int kSlotFloats = 3 * kIrrTexels + 2 * kDistTexels;   // one probe's texel gradients (RGB, mu mu2)
static_assert(kIrrTexels == 64 && kDistTexels == 256 && kWaveTerms % 64 == 0, "one lane: one irradiance texel, "
              "a column of four distance texels");

__device__ __forceinline__ uint32_t pieces_of(const uint32_t* start, const uint32_t* end, uint32_t k) {
  const uint32_t a = start[k], b = end[k];
  return b > a ? (b - a + kPieceTerms - 1) / kPieceTerms : 0u;
}

// offs[k]: the first piece of segment k (offs[K] = all pieces); poffs[k]: its
// first stored sum (segments of two or more pieces only).  One workgroup:
// contiguous runs of segments per thread, then a scan over threads.
__global__ __launch_bounds__(1024) void k_piece_offsets(const uint32_t* start, const uint32_t* end, uint32_t K,
                                                       uint32_t* offs, uint32_t* poffs) {
  __shared__ uint32_t s1[1024], s2[1024];
  const uint32_t t = threadIdx.x, per = (K + 1023) / 1024;
  const uint32_t k0 = min(K, t * per), k1 = min(K, k0 + per);
  uint32_t a1 = 0, a2 = 0;
  for (uint32_t k = k0; k < k1; k++) {
    const uint32_t n = pieces_of(start, end, k);
    a1 += n;
    a2 += n > 1 ? n : 0u;
  }
  s1[t] = a1;
  s2[t] = a2;
  for (uint32_t off = 1; off < 1024; off <<= 1) {
    __syncthreads();
    const uint32_t v1 = t >= off ? s1[t - off] : 0u, v2 = t >= off ? s2[t - off] : 0u;
    __syncthreads();
    s1[t] += v1;
    s2[t] += v2;
  }
  uint32_t b1 = s1[t] - a1, b2 = s2[t] - a2;
  for (uint32_t k = k0; k < k1; k++) {
    const uint32_t n = pieces_of(start, end, k);
    offs[k] = b1;
    poffs[k] = b2;
    b1 += n;
    b2 += n > 1 ? n : 0u;
  }
  if (t == 1023) {
    offs[K] = s1[1023];
    poffs[K] = s2[1023];
  }
}

// Index of a probe's texel gradient value s (0 .. kSlotFloats-1) in the
// gradient atlases: irradiance texel s / 3 channel s % 3, then distance
// texel (s - 192) / 2 channel (s - 192) % 2.
__device__ __forceinline__ float* slot_target(const GradSet& G, int v, int q, int s) {
  if (s < 3 * kIrrTexels) return G.irr[v] + ((size_t)q * kIrrTexels + s / 3) * 4 + s % 3;
  s -= 3 * kIrrTexels;
  return G.dist[v] + ((size_t)q * kDistTexels + s / 2) * 2 + s % 2;
}

__device__ __forceinline__ float corner_weight(int x, int x0, float f) {
  return x == x0 ? 1.0f - f : (x == x0 + 1 ? f : 0.0f);
}

// One workgroup per piece (the grid bounds the number of pieces; the rest
// return).  Probe pieces: wave w takes the piece's batches of 64 terms w,
// w + 4, w + 8, ... in order, through LDS; lane l accumulates irradiance
// texel l and distance texels (l % 16, 4 (l / 16) .. + 3); the four waves'
// sums are added in wave order.  Material pieces: thread t sums terms t,
// t + 256, ... then a fixed tree over threads.  Keys: [0, P) probes,
// [P, K) materials.
__global__ __launch_bounds__(256) void k_gather_pieces(VolumeSet vs, uint32_t P, uint32_t K, const Term* terms,
                                                       const uint32_t* idx, const uint32_t* start,
                                                       const uint32_t* end, const uint32_t* offs,
                                                       const uint32_t* poffs, float* partial, uint32_t max_partial,
                                                       GradSet G, float* g_emission) {
  __shared__ Term s_t[kPieceWaves][64];
  __shared__ float s_red[kPieceWaves * kSlotFloats];
  const uint32_t w = blockIdx.x;
  if (w >= offs[K]) return;
  uint32_t lo = 0, hi = K - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  const uint32_t k = lo, j = w - offs[k], n = offs[k + 1] - offs[k];
  const uint32_t a = start[k] + j * kPieceTerms, b = min(end[k], a + kPieceTerms);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  float* out = nullptr;   // stored sums of a segment of several pieces
  if (n > 1) {
    // a segment of n > 1 pieces has more than kPieceTerms terms, so its n <
    // 2 len / kPieceTerms and all stored pieces of a batch number below
    // 2 x batch terms / kPieceTerms = max_partial; the test keeps the write
    // inside the buffer regardless
    const uint32_t slot = poffs[k] + j;
    if (slot >= max_partial) return;
    out = partial + (size_t)slot * kSlotFloats;
  }
  if (k >= P) {
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (uint32_t i = a + t; i < b; i += 256) {
      const Term& T = terms[idx[i]];
      for (int c = 0; c < 3; c++) acc[c] += T.ge[c];
    }
    for (int c = 0; c < 3; c++) s_red[c * 256 + t] = acc[c];
    for (int half = 128; half > 0; half >>= 1) {
      __syncthreads();
      if (t < half)
        for (int c = 0; c < 3; c++) s_red[c * 256 + t] += s_red[c * 256 + t + half];
    }
    if (t < 3) {
      if (out) out[t] = s_red[t * 256];
      else g_emission[3 * (k - P) + t] += s_red[t * 256];
    }
    return;
  }
  const int xi = lane % kIrrTile, yi = lane / kIrrTile, xd = lane % kDistTile, yd0 = 4 * (lane / kDistTile);
  float ai[3] = {0.0f, 0.0f, 0.0f}, ad[4][2] = {{0.0f, 0.0f}, {0.0f, 0.0f}, {0.0f, 0.0f}, {0.0f, 0.0f}};
  for (int batch = 0; batch < kWaveTerms / 64; batch++) {
    const uint32_t b0 = a + (uint32_t)(batch * kPieceWaves + wave) * 64;
    const int cnt = b0 < b ? (int)min(64u, b - b0) : 0;
    __syncthreads();
    if (lane < cnt) s_t[wave][lane] = terms[idx[b0 + lane]];
    __syncthreads();
    for (int i = 0; i < cnt; i++) {
      const Term& T = s_t[wave][i];
      const int ix = T.fp & 255, iy = (T.fp >> 8) & 255;
      const float wb = corner_weight(xi, ix, T.ifx) * corner_weight(yi, iy, T.ify);
      for (int c = 0; c < 3; c++) ai[c] = fmaf(wb, T.ge[c], ai[c]);
      if (T.gd[0] != 0.0f || T.gd[1] != 0.0f) {
        const int dx = (T.fp >> 16) & 255, dy = T.fp >> 24;
        const float wx = corner_weight(xd, dx, T.dfx);
        for (int r = 0; r < 4; r++) {
          const float wd = wx * corner_weight(yd0 + r, dy, T.dfy);
          ad[r][0] = fmaf(wd, T.gd[0], ad[r][0]);
          ad[r][1] = fmaf(wd, T.gd[1], ad[r][1]);
        }
      }
    }
  }
  float* red = s_red + wave * kSlotFloats;
  for (int c = 0; c < 3; c++) red[lane * 3 + c] = ai[c];
  for (int r = 0; r < 4; r++)
    for (int c = 0; c < 2; c++) red[3 * kIrrTexels + ((yd0 + r) * kDistTile + xd) * 2 + c] = ad[r][c];
  __syncthreads();
  int v = 0;
  while (v + 1 < vs.n && (int)k >= vs.v[v + 1].probe_base) v++;
  const int q = (int)k - vs.v[v].probe_base;
  for (int s = t; s < kSlotFloats; s += 256) {
    float sum = s_red[s];
    for (int wv = 1; wv < kPieceWaves; wv++) sum += s_red[wv * kSlotFloats + s];
    if (out) out[s] = sum;
    else *slot_target(G, v, q, s) += sum;
  }
}

// Segments of two or more pieces: their stored sums added in piece order.
__global__ __launch_bounds__(256) void k_finish_pieces(VolumeSet vs, uint32_t P, uint32_t K, const uint32_t* offs,
                                                       const uint32_t* poffs, const float* partial,
                                                       uint32_t max_partial, GradSet G, float* g_emission) {
  const uint32_t k = blockIdx.x;
  const uint32_t n = offs[k + 1] - offs[k], p0 = poffs[k];
  if (n < 2 || p0 + n > max_partial) return;
  const int t = threadIdx.x;
  if (k >= P) {
    if (t < 3) {
      float sum = 0.0f;
      for (uint32_t j = 0; j < n; j++) sum += partial[(size_t)(p0 + j) * kSlotFloats + t];
      g_emission[3 * (k - P) + t] += sum;
    }
    return;
  }
  int v = 0;
  while (v + 1 < vs.n && (int)k >= vs.v[v + 1].probe_base) v++;
  const int q = (int)k - vs.v[v].probe_base;
  for (int s = t; s < kSlotFloats; s += 256) {
    float sum = 0.0f;
    for (uint32_t j = 0; j < n; j++) sum += partial[(size_t)(p0 + j) * kSlotFloats + s];
    *slot_target(G, v, q, s) += sum;
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
constexpr int kNormsPerVolume = 36 + 196;   // interior irradiance texels, interior distance texels

// Per volume: the inverse of each interior texel's weight sum over the
// frame's rays (0 for an empty sum), irradiance texels first.  Every probe of
// a volume traces the same rotated directions, so one row per volume.  One
// workgroup per (texel, volume): thread t sums rays t, t + 256, ..., then a
// fixed tree over lanes and waves.
__global__ __launch_bounds__(kBwdBlock) void k_blend_norms(VolumeSet prev, FrameScratch fs, float* norms) {
  __shared__ float s_part[kBwdBlock / 64];
  const int row = blockIdx.x, v = blockIdx.y, t = threadIdx.x;
  const VolumeGPU& V = prev.v[v];
  const float4* om = fs.omega + V.omega_base;
  const bool irr = row < 36;
  const float3 nt = irr ? texel_direction<kIrrTile>(row % 6 + 1, row / 6 + 1)
                        : texel_direction<kDistTile>((row - 36) % 14 + 1, (row - 36) / 14 + 1);
  float W = 0.0f;
  for (int r = t; r < V.rays; r += kBwdBlock) {
    const float4 o = om[r];
    const float c = fmaf(nt.x, o.x, fmaf(nt.y, o.y, nt.z * o.z));
    if (c > 0.0f) W += irr ? c : pow_weight(c, V);
  }
  for (int off = 32; off > 0; off >>= 1) W += __shfl_down(W, off);
  if ((t & 63) == 0) s_part[t >> 6] = W;
  __syncthreads();
  if (t == 0) {
    float sum = s_part[0];
    for (int w = 1; w < kBwdBlock / 64; w++) sum += s_part[w];
    norms[(size_t)v * kNormsPerVolume + row] = sum > 0.0f ? 1.0f / sum : 0.0f;
  }
}

// One workgroup per probe of every volume.  prev: the frame's input atlases
// and the states after its state step.
__global__ __launch_bounds__(kBwdBlock) void k_blend_backward(VolumeSet prev, FrameScratch fs, const float* norms,
                                                              GradSet Gnew, GradSet Gprev) {
  __shared__ float s_g[36][3];
  __shared__ float s_iW[36];
  __shared__ float3 s_nt[36];
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
  const float* nv = norms + (size_t)v * kNormsPerVolume;
  const int t = threadIdx.x;
  if (t < 36) {
    const int x = t % 6 + 1, y = t / 6 + 1;
    s_nt[t] = texel_direction<kIrrTile>(x, y);
    const float iW = nv[t];
    s_iW[t] = iW;
    for (int c = 0; c < 3; c++) {
      float g = folded<kIrrTile>(gi, 4, c, x, y);
      s_g[t][c] = g;
      pi[(y * kIrrTile + x) * 4 + c] += (iW > 0.0f ? ai : 1.0f) * g;
    }
  }
  if (t < 196) {
    const int x = t % 14 + 1, y = t / 14 + 1;
    // a zero weight sum keeps the texel
    const bool any = nv[36 + t] > 0.0f;
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
#pragma unroll 4
    for (int k = 0; k < 36; k++) {
      const float3 nt = s_nt[k];
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

// Rays [r0, r0 + n) of the frame (front faces only; misses and backfaces
// carry constants), 8 prev.n + 1 slots per ray at (r - r0) * (8 prev.n + 1):
// the terms of the previous-frame query at the hit, with upstream albedo x
// the ray's radiance gradient, then its emitter record (key P + material,
// ge = the radiance gradient).  Keys of empty slots: `none`.
__global__ __launch_bounds__(256) void k_shade_terms(VolumeSet prev, SceneGPU sc, FrameScratch fs, int64_t r0, int64_t n, Term* terms,
                              uint32_t* keys, uint32_t P, uint32_t none) {
  const FrameCounters& C = *fs.counters;
  const int64_t total = C.ray_base[prev.n];
  const int per = 8 * prev.n + 1;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    Term* tj = terms + j * per;
    uint32_t* kj = keys + j * per;
    for (int k = 0; k < per; k++) kj[k] = none;
    const int64_t id = r0 + j;
    if (id >= total) continue;
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
    Term E = {};
    E.ge[0] = g.x;
    E.ge[1] = g.y;
    E.ge[2] = g.z;
    tj[per - 1] = E;
    kj[per - 1] = P + (uint32_t)m;
    const float4 al = sc.albedo[m];
    // the hit in double: the ray (probe position, direction) and its
    // distance to the hit triangle's plane
    const D3 o = position_d(V, q);
    const D3 wd = sf_direction_d(r, V.rays, fs.params->R);
    const D3 va = d3(a.x, a.y, a.z), vb = d3(b.x, b.y, b.z), vc = d3(c.x, c.y, c.z);
    const D3 nn = crossd(vb - va, vc - va);
    const double td = dotd(va - o, nn) / dotd(wd, nn);
    const D3 X = o + td * wd;
    query_terms(prev, X, normalized(nn), d3(-wd.x, -wd.y, -wd.z),
                d3((double)al.x * g.x, (double)al.y * g.y, (double)al.z * g.z), tj, kj, none);
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

static inline unsigned grid_of(int64_t n, int block) {
  const int64_t b = (n + block - 1) / block;
  return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

// Bits that hold keys 0 .. none.
static inline unsigned key_bits(uint32_t none) {
  unsigned b = 1;
  while (b < 32 && (1ull << b) <= none) b++;
  return b;
}

// Onesweep radix sort at every size above one block (rocPRIM's merge-sort
// path for mid sizes is several times slower on these key widths).
using SortConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                              rocprim::default_config, 0>;

size_t adjoint_sort_bytes(int64_t max_pairs) {
  size_t bytes = 0;
  (void)rocprim::radix_sort_pairs<SortConfig>(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                              rocprim::counting_iterator<uint32_t>(0u), (uint32_t*)nullptr,
                                              (unsigned)max_pairs, 0u, 32u);
  return bytes;
}

int64_t adjoint_partial_slots(int64_t max_terms) { return 2 * (max_terms / kPieceTerms) + 2; }
size_t adjoint_slot_bytes() { return sizeof(float) * kSlotFloats; }
int adjoint_norms_per_volume() { return kNormsPerVolume; }

// Sorts the batch's nt terms by key (segments 0 .. K-1; `none` = K for empty
// slots) and adds each segment's terms into its probe's texels (keys below
// P) or its material's emission gradient (P .. K-1).
static hipError_t gather_batch(const VolumeSet& vs, const AdjointScratch& A, int64_t nt, uint32_t P, uint32_t K,
                               const GradSet& G, float* g_emission, hipStream_t s) {
  size_t bytes = A.sort_bytes;
  hipError_t e = rocprim::radix_sort_pairs<SortConfig>(A.sort_temp, bytes, (const uint32_t*)A.keys[0], A.keys[1],
                                                       rocprim::counting_iterator<uint32_t>(0u), A.idx, (unsigned)nt,
                                                       0u, key_bits(K), s);
  if (e != hipSuccess) return e;
  irf_launch(k_fill_words, dim3(grid_of(K, 256)), dim3(256), 0, s, A.seg_start, 0u, (int64_t)K);
  irf_launch(k_fill_words, dim3(grid_of(K, 256)), dim3(256), 0, s, A.seg_end, 0u, (int64_t)K);
  irf_launch(k_segments, dim3(grid_of(nt, 256)), dim3(256), 0, s, (const uint32_t*)A.keys[1], nt, K, A.seg_start,
             A.seg_end);
  irf_launch(k_piece_offsets, dim3(1), dim3(1024), 0, s, (const uint32_t*)A.seg_start, (const uint32_t*)A.seg_end, K,
             A.offs, A.poffs);
  const int64_t grid = (nt + kPieceTerms - 1) / kPieceTerms + K;
  irf_launch(k_gather_pieces, dim3((unsigned)grid), dim3(256), 0, s, vs, P, K, (const Term*)A.terms,
             (const uint32_t*)A.idx, (const uint32_t*)A.seg_start, (const uint32_t*)A.seg_end,
             (const uint32_t*)A.offs, (const uint32_t*)A.poffs, A.partial, (uint32_t)A.max_partial, G, g_emission);
  irf_launch(k_finish_pieces, dim3(K), dim3(256), 0, s, vs, P, K, (const uint32_t*)A.offs, (const uint32_t*)A.poffs,
             (const float*)A.partial, (uint32_t)A.max_partial, G, g_emission);
  return hipSuccess;
}

hipError_t launch_query_backward(const VolumeSet& vs, const float* pos, const float* nrm, const float* view,
                                 int64_t n, const float* gout, const GradSet& G, const AdjointScratch& A,
                                 hipStream_t s) {
  uint32_t P = 0;
  for (int v = 0; v < vs.n; v++) P += (uint32_t)vs.v[v].n_probes;
  const int per = 8 * vs.n;
  const int64_t chunk = A.max_terms / per;
  if (n == 0 || P == 0 || chunk == 0) return hipSuccess;
  for (int64_t i0 = 0; i0 < n; i0 += chunk) {
    const int64_t m = n - i0 < chunk ? n - i0 : chunk;
    irf_launch(k_query_terms, dim3(grid_of(m, 256)), dim3(256), 0, s, vs, pos, nrm, view, i0, m, gout,
               (Term*)A.terms, A.keys[0], P);
    hipError_t e = gather_batch(vs, A, m * per, P, P, G, nullptr, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_update_backward(const VolumeSet& prev, SceneGPU sc, FrameScratch fs, const GradSet& Gnew,
                                  const GradSet& Gprev, float* g_emission, int n_materials, int64_t n_rays,
                                  const AdjointScratch& A, hipStream_t s) {
  uint32_t P = 0;
  for (int v = 0; v < prev.n; v++) P += (uint32_t)prev.v[v].n_probes;
  if (P == 0) return hipSuccess;
  irf_launch(k_blend_norms, dim3(kNormsPerVolume, prev.n), dim3(kBwdBlock), 0, s, prev, fs, A.norms);
  irf_launch(k_blend_backward, dim3(P), dim3(kBwdBlock), 0, s, prev, fs, (const float*)A.norms, Gnew, Gprev);
  const int per = 8 * prev.n + 1;
  const int64_t chunk = A.max_terms / per;
  if (n_rays > fs.max_rays) n_rays = fs.max_rays;
  if (n_rays <= 0 || chunk == 0) return hipSuccess;
  const uint32_t K = P + (uint32_t)n_materials;
  for (int64_t r0 = 0; r0 < n_rays; r0 += chunk) {
    const int64_t m = n_rays - r0 < chunk ? n_rays - r0 : chunk;
    irf_launch(k_shade_terms, dim3(grid_of(m, 256)), dim3(256), 0, s, prev, sc, fs, r0, m, (Term*)A.terms, A.keys[0],
               P, K);
    hipError_t e = gather_batch(prev, A, m * per, P, K, Gprev, g_emission, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace irf
