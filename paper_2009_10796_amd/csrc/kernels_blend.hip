// The blend of the probe update as a GEMM on the matrix cores.
//
// Eq. U, read as a normalised weighted average (Section "Probe Update"), is
// for every probe the same contraction over rays:
//   new_E[texel][c]  = sum_r W_E[texel][r] L[r][c]      / sum_r W_E[texel][r]
//   new_D[texel][j]  = sum_r W_D[texel][r] d[r]^(j+1)   / sum_r W_D[texel][r]
// with W_E = max(0, n.w) and W_D = max(0, n.w)^p shared by all probes of a
// volume (one rotation per frame).  k_frame_begin builds W once per frame (rows:
// 36 irradiance interior texels padded to 48, then 196 distance interior
// texels padded to 208) and the reciprocal row sums of the *stored* weights,
// so a constant radiance is reproduced exactly whatever the input precision.
// k_blend_mma multiplies W by the rays of 8 probes at a time:
//   columns  0..7 R, 8..15 G, 16..23 B of probes 0..7 (24..31 zero),
//   columns 32..39  d, 40..47 d^2 of probes 0..7,
// with v_mfma_f32_16x16x4_f32 (float32 inputs) or v_mfma_f32_16x16x32_{bf16,f16}
// (16-bit inputs), float32 accumulation.  The epilogue normalises, applies the
// hysteresis (0 for Newly states; for irradiance the stored encoding and the
// per-texel thresholds of the convergence sections) and writes each texel and
// the border cells that repeat it; the first row slice of each probe block
// then promotes its Newly probes.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace irf {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int kPB = 8;            // probes per workgroup
// Rays per LDS chunk: 64, a B tile of 12.25 KiB (float32) or 6.75 KiB
// (16-bit), so a compute unit holds many work items at once.  On the terrain
// cascades the blend took 130-170 us (float32) and 88-105 us (16-bit) with
// 256-ray chunks, 78-95 and 51-75 us with 64.  The products run over the rays
// in the same order whatever the chunk, so results do not change.
constexpr int kKC = 64;
constexpr int kBlendMmaBlock = 256;
constexpr int kBfStride = 49;     // float32 B tile: [k][48 + 1]
constexpr int kBtStride = 64 + 8; // 16-bit B tile: [col][64 + 8]

template <int MODE>
struct Mma;

// float32 inputs: v_mfma_f32_16x16x4_f32.  A fragment: lane l holds
// W[row0 + l%16][k0 + l/16]; B fragment: B[k0 + l/16][col0 + l%16].
template <>
struct Mma<IRF_BLEND_F32> {
  static constexpr int KSTEP = 4;
  static constexpr int KB = 16;    // k-steps whose A fragments are loaded together
  typedef float A;
  __device__ static A load_a(const char* wbase, int row_tile, int k, int N, int lane) {
    const int kk = min(k + lane / 16, N - 1);   // rays past N: any finite weight (their B is zero)
    return ((const float*)wbase)[(size_t)kk * kRows + row_tile * 16 + lane % 16];
  }
  __device__ static A load_b(const char* lds, int col_base, int k, int lane) {
    return ((const float*)lds)[(k + lane / 16) * kBfStride + col_base + lane % 16];
  }
  __device__ static v4f mma(A a, A b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

// 16-bit inputs: v_mfma_f32_16x16x32_{bf16,f16}.  A fragment: lane l holds
// W[row0 + l%16][k0 + 8(l/16) .. +7]; B fragment: B[k0 + 8(l/16) .. +7][col0 + l%16].
template <>
struct Mma<IRF_BLEND_BF16> {
  static constexpr int KSTEP = 32;
  static constexpr int KB = 2;     // k-steps whose A fragments are loaded together (one 64-ray chunk)
  typedef v8bf A;
  __device__ static A load_a(const char* wbase, int row_tile, int k, int N, int lane) {
    const int kk = min(k + 8 * (lane / 16), N - 8);   // rays past N: any finite weights (their B is zero)
    return *(const v8bf*)((const __bf16*)wbase + (size_t)(row_tile * 16 + lane % 16) * N + kk);
  }
  __device__ static A load_b(const char* lds, int col_base, int k, int lane) {
    return *(const v8bf*)((const __bf16*)lds + (col_base + lane % 16) * kBtStride + k + 8 * (lane / 16));
  }
  __device__ static v4f mma(A a, A b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

template <>
struct Mma<IRF_BLEND_F16> {
  static constexpr int KSTEP = 32;
  static constexpr int KB = 2;     // k-steps whose A fragments are loaded together (one 64-ray chunk)
  typedef v8h A;
  __device__ static A load_a(const char* wbase, int row_tile, int k, int N, int lane) {
    const int kk = min(k + 8 * (lane / 16), N - 8);   // rays past N: any finite weights (their B is zero)
    return *(const v8h*)((const _Float16*)wbase + (size_t)(row_tile * 16 + lane % 16) * N + kk);
  }
  __device__ static A load_b(const char* lds, int col_base, int k, int lane) {
    return *(const v8h*)((const _Float16*)lds + (col_base + lane % 16) * kBtStride + k + 8 * (lane / 16));
  }
  __device__ static v4f mma(A a, A b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

template <int MODE>
__device__ __forceinline__ void store_b(void* lds, int k, int col, float x) {
  if constexpr (MODE == IRF_BLEND_F32) {
    ((float*)lds)[k * kBfStride + col] = x;
  } else if constexpr (MODE == IRF_BLEND_BF16) {
    ((__bf16*)lds)[col * kBtStride + k] = (__bf16)x;
  } else {
    ((_Float16*)lds)[col * kBtStride + k] = (_Float16)x;
  }
}

// One irradiance texel (RGB, 4th channel 0), float4 or half4.
__device__ __forceinline__ void store_irr4(const VolumeGPU& V, int q, int x, int y, float3 val) {
  int j = q * kIrrTexels + y * kIrrTile + x;
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
}

__device__ __forceinline__ void store_dist(const VolumeGPU& V, int q, int x, int y, int c, float val) {
  int j = q * kDistTexels + y * kDistTile + x;
  if (V.atlas_f16) ((_Float16*)V.dist)[2 * j + c] = (_Float16)val;
  else ((float*)V.dist)[2 * j + c] = val;
}

__device__ __forceinline__ float load_ch(const VolumeGPU& V, bool irr, int q, int x, int y, int c) {
  if (irr) {
    int j = q * kIrrTexels + y * kIrrTile + x;
    return V.atlas_f16 ? (float)((const _Float16*)V.irr)[4 * j + c] : ((const float*)V.irr)[4 * j + c];
  }
  int j = q * kDistTexels + y * kDistTile + x;
  return V.atlas_f16 ? (float)((const _Float16*)V.dist)[2 * j + c] : ((const float*)V.dist)[2 * j + c];
}

// One row tile's texels from its accumulators: acc[0] (and acc[1] for
// irradiance rows) hold rows rt*16 + 4*(lane/16) + r of column col_base + lane%16.
// The old texels come prefetched (OLD) or are loaded here.
template <int MODE, bool OLD>
__device__ __forceinline__ void tile_epilogue(const VolumeGPU& V, int rt, int lane, int np, const int* s_q,
                                              const bool* s_fresh, const v4f* acc, const float* sc,
                                              const float3* old_irr, const float* old_dist) {
  if (rt < 3) {
    // irradiance rows: lane%16 = p < 8 holds R (tile 0) and B (tile 1) of
    // probe p; G comes from 8 lanes up.  The whole texel is updated at once
    // (encoding, per-texel hysteresis) by that lane.
    const int p = lane % 16;
    float gch[4];
#pragma unroll
    for (int r = 0; r < 4; r++) gch[r] = __shfl_down(acc[0][r], 8, 16);
    if (p >= 8 || p >= np) return;
    const int q = s_q[p];
    const float a = s_fresh[p] ? 0.0f : V.alpha_irr;
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int row = rt * 16 + 4 * (lane / 16) + r;
      if (sc[r] == 0.0f) continue;   // padding row, or no ray with positive weight: keep the texel
      const int x = row % 6 + 1, y = row / 6 + 1;
      const float3 old = OLD ? old_irr[r] : load_irr(V, q * kIrrTexels + y * kIrrTile + x);
      const float3 val = irr_texel_update(V, a, old, f3(acc[0][r] * sc[r], gch[r] * sc[r], acc[1][r] * sc[r]));
      store_irr4(V, q, x, y, val);
      if (y == 1) store_irr4(V, q, 7 - x, 0, val);
      if (y == 6) store_irr4(V, q, 7 - x, 7, val);
      if (x == 1) store_irr4(V, q, 0, 7 - y, val);
      if (x == 6) store_irr4(V, q, 7, 7 - y, val);
      if (x == 6 && y == 6) store_irr4(V, q, 0, 0, val);
      if (x == 1 && y == 6) store_irr4(V, q, 7, 0, val);
      if (x == 6 && y == 1) store_irr4(V, q, 0, 7, val);
      if (x == 1 && y == 1) store_irr4(V, q, 7, 7, val);
    }
    return;
  }
  // distance rows: one column tile, d of probe p at 32 + p, d^2 at 40 + p
  const int col = 32 + lane % 16;
  const int p = col - 32 < 8 ? col - 32 : col - 40;
  const int c = col - 32 < 8 ? 0 : 1;
  if (p >= np) return;
  const int q = s_q[p];
  const float a = s_fresh[p] ? 0.0f : V.alpha_dist;
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int row = rt * 16 + 4 * (lane / 16) + r;
    if (sc[r] == 0.0f) continue;
    const float nv = acc[0][r] * sc[r];
    const int rr = row - kIrrRows;
    const int x = rr % 14 + 1, y = rr / 14 + 1;
    const float old = OLD ? old_dist[r] : load_ch(V, false, q, x, y, c);
    const float val = fmaf(a, old, (1.0f - a) * nv);   // one rounding order in every kernel shape
    store_dist(V, q, x, y, c, val);
    if (y == 1) store_dist(V, q, 15 - x, 0, c, val);
    if (y == 14) store_dist(V, q, 15 - x, 15, c, val);
    if (x == 1) store_dist(V, q, 0, 15 - y, c, val);
    if (x == 14) store_dist(V, q, 15, 15 - y, c, val);
    if (x == 14 && y == 14) store_dist(V, q, 0, 0, c, val);
    if (x == 1 && y == 14) store_dist(V, q, 15, 0, c, val);
    if (x == 14 && y == 1) store_dist(V, q, 0, 15, c, val);
    if (x == 1 && y == 1) store_dist(V, q, 15, 15, c, val);
  }
}

// One work item: row split `split` of probe block `pblock` of volume v.  RS
// workgroups share a probe block; the workgroup owns row tiles split,
// split + RS, ... and wave w of it the w-th, (w + 4)-th, ... of those
// (16 / (4 RS) tiles per wave).
template <int MODE, int RS>
__device__ __forceinline__ void blend_item(const VolumeSet& vs, const FrameScratch& fs, const FrameCounters& C, int v,
                                           int pblock, int split, char* lds, int* s_q, bool* s_fresh) {
  constexpr int kTiles = 16 / (4 * RS);
  static_assert(kTiles * 4 * RS == 16, "the row split divides the 16 row tiles over 4 waves");
  const VolumeGPU& V = vs.v[v];
  const int count = C.slot_base[v + 1] - C.slot_base[v];
  const int slot0 = pblock * kPB;
  const int np = min(kPB, count - slot0);
  const int N = V.rays;
  if (threadIdx.x < kPB) {
    const int gslot = C.slot_base[v] + slot0 + threadIdx.x;
    const bool real = threadIdx.x < np;
    s_q[threadIdx.x] = real ? fs.active[gslot] - V.probe_base : -1;
    s_fresh[threadIdx.x] = real && fs.probe_pos[gslot].w != 0.0f;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int rt[kTiles];
#pragma unroll
  for (int i = 0; i < kTiles; i++) rt[i] = split + RS * (wave + 4 * i);
  const float4* rays = fs.rays + C.ray_base[v] + (int64_t)slot0 * N;
  typedef Mma<MODE> M;
  constexpr int kRound = M::KB * M::KSTEP;   // rays per round of A fragments
  constexpr int kRounds = kKC / kRound;      // rounds per chunk
  constexpr int kStage = kPB * kKC / kBlendMmaBlock;   // rays each thread stages per chunk
  static_assert(kKC % kRound == 0 && (kPB * kKC) % kBlendMmaBlock == 0, "whole rounds and stages per chunk");
  const char* wbase = (const char*)fs.weights + V.weight_base;
  // Every global read that does not depend on another is issued up front, so
  // that one memory latency, not four, precedes the products: the first
  // tile's A fragments and this thread's rays for the chunk (registers until
  // the LDS is free), the rows' reciprocal sums; then, once the probe slots
  // are known, the epilogue's old texels.  A later tile's A fragments are
  // loaded as the previous tile's products issue.
  typename M::A a[kRounds * M::KB];
  float4 rv[kStage];
  auto load_a = [&](int tile, int kc) {
    const int kn = min(kKC, N - kc);
    const int rounds = (kn + kRound - 1) / kRound;
#pragma unroll
    for (int r0 = 0; r0 < kRounds; r0++)
      if (r0 < rounds)
#pragma unroll
        for (int j = 0; j < M::KB; j++)
          a[r0 * M::KB + j] = M::load_a(wbase, tile, kc + r0 * kRound + j * M::KSTEP, N, lane);
  };
  auto load_rays = [&](int kc) {
    const int kn = min(kKC, N - kc);
#pragma unroll
    for (int i = 0; i < kStage; i++) {
      const int e = (int)threadIdx.x + i * kBlendMmaBlock;
      const int p = e / kn, k = e - p * kn;
      rv[i] = e < kPB * kn && p < np ? rays[(int64_t)p * N + kc + k] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
  };
  load_a(rt[0], 0);
  load_rays(0);
  const float* inv = fs.inv_row_sum + v * kRows;
  float sc[kTiles][4];
#pragma unroll
  for (int i = 0; i < kTiles; i++)
#pragma unroll
    for (int r = 0; r < 4; r++) sc[i][r] = inv[rt[i] * 16 + 4 * (lane / 16) + r];
  __syncthreads();   // s_q / s_fresh
  // old texels: irradiance lanes p < 8 hold rows 4 (lane / 16) + r of probe
  // p; distance lanes channel c of probe p for the same rows (prefetched for
  // up to two tiles per wave; four would spill registers)
  constexpr bool kOld = kTiles <= 2;
  float3 old_irr[kTiles][4];
  float old_dist[kTiles][4];
  if (kOld) {
    const int p = lane % 16;
    const int pd = p < 8 ? p : p - 8, cd = p < 8 ? 0 : 1;
#pragma unroll
    for (int i = 0; i < kTiles; i++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = rt[i] * 16 + 4 * (lane / 16) + r;
        old_irr[i][r] = f3(0.0f, 0.0f, 0.0f);
        old_dist[i][r] = 0.0f;
        if (rt[i] < 3) {
          if (p < np && row < 36)
            old_irr[i][r] = load_irr(V, s_q[p] * kIrrTexels + (row / 6 + 1) * kIrrTile + row % 6 + 1);
        } else {
          const int rr = row - kIrrRows;
          if (pd < np && rr < 196) old_dist[i][r] = load_ch(V, false, s_q[pd], rr % 14 + 1, rr / 14 + 1, cd);
        }
      }
  }
  v4f acc[kTiles][2];
#pragma unroll
  for (int i = 0; i < kTiles; i++) acc[i][0] = acc[i][1] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  for (int kc = 0; kc < N; kc += kKC) {
    if (kc > 0) {
      load_a(rt[0], kc);
      load_rays(kc);
    }
    const int kn = min(kKC, N - kc);
    // the products run over whole rounds with no per-step guard (a guarded
    // step splits the accumulator chain into basic blocks); rays from kn to
    // the round's end are zero in B
    const int rounds = (kn + kRound - 1) / kRound;
    const int kpad = rounds * kRound;
    __syncthreads();   // the previous chunk's products are done with the LDS
    for (int e = threadIdx.x; e < kPB * (kpad - kn); e += kBlendMmaBlock) {
      const int p = e / (kpad - kn), k = kn + e % (kpad - kn);
#pragma unroll
      for (int c = 0; c < 6; c++)
        if (c != 3) store_b<MODE>(lds, k, 8 * c + p, 0.0f);
    }
#pragma unroll
    for (int i = 0; i < kStage; i++) {
      const int e = (int)threadIdx.x + i * kBlendMmaBlock;
      if (e >= kPB * kn) continue;
      const int p = e / kn, k = e - p * kn;
      const float4 r = rv[i];
      // columns: R of probe p at p, G at 8 + p, B at 16 + p (24..31 stay
      // zero from the kernel's start), so one lane of the epilogue holds R and
      // B of a texel and G is 8 lanes up
      store_b<MODE>(lds, k, p, r.x);
      store_b<MODE>(lds, k, 8 + p, r.y);
      store_b<MODE>(lds, k, 16 + p, r.z);
      store_b<MODE>(lds, k, 32 + p, r.w);
      store_b<MODE>(lds, k, 40 + p, r.w * r.w);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kTiles; i++) {
      if (i > 0) load_a(rt[i], kc);
      if (rt[i] < 3) {
        // irradiance rows: two column tiles (R, G | B, 0), chains interleaved
#pragma unroll
        for (int r0 = 0; r0 < kRounds; r0++)
          if (r0 < rounds)
#pragma unroll
            for (int j = 0; j < M::KB; j++) {
              const int k = r0 * kRound + j * M::KSTEP;
              acc[i][0] = M::mma(a[r0 * M::KB + j], M::load_b(lds, 0, k, lane), acc[i][0]);
              acc[i][1] = M::mma(a[r0 * M::KB + j], M::load_b(lds, 16, k, lane), acc[i][1]);
            }
      } else {
        // distance rows: one column tile (d, d^2)
#pragma unroll
        for (int r0 = 0; r0 < kRounds; r0++)
          if (r0 < rounds)
#pragma unroll
            for (int j = 0; j < M::KB; j++)
              acc[i][0] =
                  M::mma(a[r0 * M::KB + j], M::load_b(lds, 32, r0 * kRound + j * M::KSTEP, lane), acc[i][0]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kTiles; i++)
    tile_epilogue<MODE, kOld>(V, rt[i], lane, np, s_q, s_fresh, acc[i], sc[i], old_irr[i], old_dist[i]);
  // Newly states are promoted once blended (the Newly flag of this frame is
  // the slot's, so no workgroup reads the state itself)
  if (split == 0 && threadIdx.x < np && s_fresh[threadIdx.x]) {
    const int q = s_q[threadIdx.x];
    V.states[q] = V.states[q] == IRF_NEWLY_AWAKE ? IRF_AWAKE : IRF_VIGILANT;
  }
}

// Persistent over work items (probe block x row split) of every volume whose
// blend mode is MODE.  Workgroups are dispatched to the 8 XCDs round robin
// (XCD = workgroup id mod 8) and the grid is a multiple of 8, so item wi runs
// on XCD wi mod 8; item wi is split (wi / 8) mod RS of probe block
// (wi / (8 RS)) * 8 + wi mod 8, which puts the RS items of a block -- the same
// rays staged RS times -- on one XCD, and on one L2.
template <int MODE, int RS>
__global__ __launch_bounds__(kBlendMmaBlock) void k_blend_mma(VolumeSet vs, FrameScratch fs) {
  constexpr int LDS_BYTES = MODE == IRF_BLEND_F32 ? kKC * kBfStride * 4 : 48 * kBtStride * 2;
  __shared__ __attribute__((aligned(16))) char lds[LDS_BYTES];
  __shared__ int s_q[kPB];
  __shared__ bool s_fresh[kPB];
  const FrameCounters& C = *fs.counters;
  int block_base[IRF_MAX_VOLUMES + 1];
  block_base[0] = 0;
  for (int v = 0; v < vs.n; v++) {
    int count = vs.v[v].blend == MODE ? C.slot_base[v + 1] - C.slot_base[v] : 0;
    block_base[v + 1] = block_base[v] + (count + kPB - 1) / kPB;
  }
  // B columns 24..31 (the irradiance tiles' unused half) are zero for the
  // whole kernel; the staging never writes them
  for (int e = threadIdx.x; e < kKC * 8; e += kBlendMmaBlock) store_b<MODE>(lds, e / 8, 24 + e % 8, 0.0f);
  const int blocks = block_base[vs.n];
  const int items = (blocks + 7) / 8 * 8 * RS;
  for (int wi = blockIdx.x; wi < items; wi += gridDim.x) {
    const int b = (wi / (8 * RS)) * 8 + (wi & 7);
    if (b >= blocks) continue;
    int v = 0;
    while (v + 1 < vs.n && b >= block_base[v + 1]) v++;
    __syncthreads();   // the previous item's epilogue has finished with s_q / s_fresh
    blend_item<MODE, RS>(vs, fs, C, v, b - block_base[v], (wi / 8) % RS, lds, s_q, s_fresh);
  }
}

template <int MODE>
static void launch_mode(const VolumeSet& vs, FrameScratch fs, unsigned grid, int rsplit, hipStream_t s) {
  if (rsplit == 1)
    irf_launch(k_blend_mma<MODE, 1>, dim3(grid), dim3(kBlendMmaBlock), 0, s, vs, fs);
  else if (rsplit == 2)
    irf_launch(k_blend_mma<MODE, 2>, dim3(grid), dim3(kBlendMmaBlock), 0, s, vs, fs);
  else
    irf_launch(k_blend_mma<MODE, 4>, dim3(grid), dim3(kBlendMmaBlock), 0, s, vs, fs);
}

void launch_blend_mma(const VolumeSet& vs, FrameScratch fs, int grid, int rsplit, hipStream_t s) {
  if (rsplit != 1 && rsplit != 2) rsplit = 4;
  bool mode_present[3] = {false, false, false};
  int full = 0;
  for (int v = 0; v < vs.n; v++) {
    full += (vs.v[v].n_probes + kPB - 1) / kPB * rsplit;
    if (vs.v[v].blend <= IRF_BLEND_F16) mode_present[vs.v[v].blend] = true;
  }
  if (full == 0) return;
  // items of probe blocks rounded up to groups of 8 (see k_blend_mma); a grid
  // that is a multiple of 8 keeps each block's row splits on one XCD
  full = (full + 8 * rsplit - 1) / (8 * rsplit) * (8 * rsplit);
  const int want = grid > 0 && grid < full ? grid : full;
  const unsigned g = (unsigned)((want + 7) / 8 * 8);
  if (mode_present[IRF_BLEND_F32]) launch_mode<IRF_BLEND_F32>(vs, fs, g, rsplit, s);
  if (mode_present[IRF_BLEND_BF16]) launch_mode<IRF_BLEND_BF16>(vs, fs, g, rsplit, s);
  if (mode_present[IRF_BLEND_F16]) launch_mode<IRF_BLEND_F16>(vs, fs, g, rsplit, s);
}

}  // namespace irf
