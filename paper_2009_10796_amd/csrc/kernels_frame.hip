// Start of an update frame, in one launch (k_frame_begin):
//
//  directions   the frame's rotated spherical-Fibonacci ray directions (one
//               rotation shared by every probe of every volume, Section
//               "Probe Update"), and the frame's parameters (rotation, lights)
//  weights      rows of the matrix-core blend's weight matrix: for interior
//               texel direction n and ray direction w, max(0, n.w) for the
//               irradiance rows and max(0, n.w)^p for the distance rows, in
//               the volume's input format, and the reciprocal of each row's
//               float32 sum of the stored weights
//  compaction   the per-frame state step (dynamic objects wake sleeping
//               probes near them and put awake ones that are no longer near
//               back to sleep, Section "Probe States") and the list of active
//               probes, packed across volumes in probe order, with each
//               slot's probe position
//
// The three parts read nothing the others write, so they share one grid:
// x-blocks [0, dir_blocks) directions, then weight_rows weight rows, then one
// compaction workgroup (blockIdx.y = volume; compaction at y = 0 only).  Past
// kSmallProbes probes the compaction runs as two kernels (per-workgroup
// counts, then an ordered scatter) launched before k_frame_begin.
#include <hip/hip_runtime.h>

#include <cstring>

#include "device_common.h"

namespace irf {

constexpr int kBeginBlock = 1024;                          // >= the largest ray count: one pass per row
constexpr int kPerThread = 4;                              // probes per thread, one-workgroup compaction
constexpr int kSmallProbes = kBeginBlock * kPerThread;     // 4096

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

// State step of probe q; returns the stepped state.
__device__ __forceinline__ uint8_t step_state(const VolumeGPU& V, ObjectBoxes ob, int q) {
  uint8_t st = V.states[q];
  if (ob.n > 0 && (st == IRF_SLEEPING || st == IRF_AWAKE)) {
    bool near = near_dynamic(V, ob, probe_position(V, q));
    uint8_t ns = st;
    if (st == IRF_SLEEPING && near) ns = IRF_NEWLY_AWAKE;
    if (st == IRF_AWAKE && !near) ns = IRF_SLEEPING;
    if (ns != st) V.states[q] = ns;
    st = ns;
  }
  return st;
}

__device__ __forceinline__ int volume_of_probe(const VolumeSet& vs, int g) {
  int v = 0;
  while (v + 1 < vs.n && g >= vs.v[v + 1].probe_base) v++;
  return v;
}

__device__ __forceinline__ bool newly(uint8_t s) { return s == IRF_NEWLY_AWAKE || s == IRF_NEWLY_VIGILANT; }

// Slot of an active probe: its global id, position and whether it is Newly
// (the blend then takes no hysteresis and promotes it).
__device__ __forceinline__ void write_slot(const VolumeSet& vs, const FrameScratch& fs, int slot, int v, int q,
                                           bool fresh) {
  const VolumeGPU& V = vs.v[v];
  fs.active[slot] = V.probe_base + q;
  const float3 P = probe_position(V, q);
  fs.probe_pos[slot] = make_float4(P.x, P.y, P.z, fresh ? 1.0f : 0.0f);
}

// Counters of the frame from the active probes per volume.
__device__ __forceinline__ void write_counters(const VolumeSet& vs, const FrameScratch& fs, const int* slot_base) {
  FrameCounters* C = fs.counters;
  int64_t rays = 0;
  for (int u = 0; u < vs.n; u++) {
    C->slot_base[u] = slot_base[u];
    C->ray_base[u] = rays;
    rays += (int64_t)(slot_base[u + 1] - slot_base[u]) * vs.v[u].rays;
  }
  C->slot_base[vs.n] = slot_base[vs.n];
  C->ray_base[vs.n] = rays;
  for (int r = 0; r < kTaskRegions; r++) C->task_count[r] = 0;
}

// Inclusive prefix sum over the workgroup (kBeginBlock threads); `total`
// receives the sum of all.
__device__ __forceinline__ int block_scan(int x, int* s_wave, int& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kBeginBlock / 64; w++) {
    int t = s_wave[w];
    before += w < wave ? t : 0;
    all += t;
  }
  total = all;
  return x + before;
}

// One workgroup: state step and ordered active list of all probes (at most
// kSmallProbes).  Thread t owns the consecutive probes [t*per, (t+1)*per) of
// the concatenated probe space, so thread order is probe order.
__device__ void compact_small(const FrameBegin& a) {
  __shared__ int s_wave[kBeginBlock / 64];
  __shared__ int s_slot[IRF_MAX_VOLUMES + 1];
  const VolumeSet& vs = a.vs;
  const int P = a.total_probes;
  const int per = (P + kBeginBlock - 1) / kBeginBlock;
  const int g0 = threadIdx.x * per;
  uint32_t bits = 0, fresh = 0;
  int v = g0 < P ? volume_of_probe(vs, g0) : 0;
  for (int j = 0; j < per; j++) {
    const int g = g0 + j;
    if (g >= P) break;
    while (v + 1 < vs.n && g >= vs.v[v + 1].probe_base) v++;
    const uint8_t st = step_state(vs.v[v], a.ob, g - vs.v[v].probe_base);
    bits |= (uint32_t)active_state(st) << j;
    fresh |= (uint32_t)newly(st) << j;
  }
  int total;
  const int incl = block_scan(__popc(bits), s_wave, total);
  const int base = incl - __popc(bits);
  if (threadIdx.x == 0)
    for (int u = 0; u <= vs.n; u++) s_slot[u] = total;
  __syncthreads();
  // slot base of each volume: active probes before its first probe
  for (int u = 0; u < vs.n; u++) {
    const int pb = vs.v[u].probe_base;
    if (pb >= g0 && pb < g0 + per && pb < P) s_slot[u] = base + __popc(bits & ((1u << (pb - g0)) - 1u));
  }
  v = g0 < P ? volume_of_probe(vs, g0) : 0;
  int slot = base;
  for (int j = 0; j < per; j++) {
    if (!(bits >> j & 1u)) continue;
    const int g = g0 + j;
    while (v + 1 < vs.n && g >= vs.v[v + 1].probe_base) v++;
    write_slot(vs, a.fs, slot++, v, g - vs.v[v].probe_base, fresh >> j & 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) write_counters(vs, a.fs, s_slot);
}

__device__ __forceinline__ float round_to(float w, int mode) {
  if (mode == IRF_BLEND_BF16) return (float)(__bf16)w;
  if (mode == IRF_BLEND_F16) return (float)(_Float16)w;
  return w;
}

// Direction of weight row `row` (irradiance rows first), false for padding.
__device__ __forceinline__ bool row_direction(int row, float3& n) {
  if (row < kIrrRows) {
    if (row >= 36) return false;
    n = texel_direction<kIrrTile>(row % 6 + 1, row / 6 + 1);
    return true;
  }
  int r = row - kIrrRows;
  if (r >= 196) return false;
  n = texel_direction<kDistTile>(r % 14 + 1, r / 14 + 1);
  return true;
}

// Weight rows of volume v over all rays (ray directions recomputed here:
// the same function of (ray, rotation) as the direction table).  A workgroup
// holds 16 / row_waves rows, each on row_waves consecutive waves, so short
// rows (few rays) share a workgroup instead of leaving most of it idle.
__device__ void weight_rows(const FrameBegin& a, int v, int block) {
  __shared__ float part[kBeginBlock / 64];
  const VolumeGPU& V = a.vs.v[v];
  if (V.blend == IRF_BLEND_F32_VALU) return;
  const FrameScratch& fs = a.fs;
  const int N = V.rays;
  const int per_row = a.row_waves * 64;                 // lanes of one row
  const int rows_here = kBeginBlock / per_row;          // rows of this workgroup
  const int sub = threadIdx.x / per_row;
  const int row = block * rows_here + sub;
  const bool live = sub < rows_here && row < kRows;
  float3 n = f3(0.0f, 0.0f, 0.0f);
  const bool real = live && row_direction(row, n);
  float sum = 0.0f;
  char* base = (char*)fs.weights + V.weight_base;
  if (live) {
    for (int k = threadIdx.x - sub * per_row; k < N; k += per_row) {
      float w = 0.0f;
      if (real) {
        const float3 o = sf_direction(k, N, a.p.R);
        const float c = fmaf(n.x, o.x, fmaf(n.y, o.y, n.z * o.z));
        w = c > 0.0f ? (row < kIrrRows ? c : pow_weight(c, V)) : 0.0f;
      }
      w = round_to(w, V.blend);
      sum += w;
      if (V.blend == IRF_BLEND_F32) {
        ((float*)base)[(size_t)k * kRows + row] = w;               // [k][row]
      } else if (V.blend == IRF_BLEND_BF16) {
        ((__bf16*)base)[(size_t)row * N + k] = (__bf16)w;          // [row][k]
      } else {
        ((_Float16*)base)[(size_t)row * N + k] = (_Float16)w;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (live && threadIdx.x == sub * per_row) {
    float t = 0.0f;
    for (int w = 0; w < a.row_waves; w++) t += part[sub * a.row_waves + w];
    fs.inv_row_sum[v * kRows + row] = t > 0.0f ? 1.0f / t : 0.0f;
  }
}

static_assert(sizeof(FrameBegin) <= 4096, "the frame-start argument block must fit the 4 KiB kernel-argument limit");

__global__ __launch_bounds__(kBeginBlock) void k_frame_begin(FrameBegin a) {
  const int v = blockIdx.y;
  if (v >= a.vs.n) return;
  const int x = blockIdx.x;
  if (x < a.dir_blocks) {
    if (x == 0 && v == 0 && threadIdx.x == 0) *a.fs.params = a.p;
    const VolumeGPU& V = a.vs.v[v];
    const int r = x * kBeginBlock + threadIdx.x;
    if (r >= V.rays) return;
    const float3 w = sf_direction(r, V.rays, a.p.R);
    a.fs.omega[V.omega_base + r] = make_float4(w.x, w.y, w.z, 0.0f);
  } else if (x < a.dir_blocks + a.weight_rows) {
    weight_rows(a, v, x - a.dir_blocks);
  } else if (v == 0 && a.compact) {
    compact_small(a);
  }
}

// ---- compaction in two passes (more than kSmallProbes probes)

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

// Pass 1: state step and the number of active probes of each workgroup.
__global__ __launch_bounds__(kCompactBlock) void k_state_count(VolumeSet vs, ObjectBoxes ob, CompactArgs A,
                                                                FrameScratch fs) {
  __shared__ int wave_tot[kCompactBlock / 64];
  const int b = blockIdx.x;
  const int v = compact_volume(A, vs.n, b);
  const VolumeGPU& V = vs.v[v];
  const int q = (b - A.block_base[v]) * kCompactBlock + threadIdx.x;
  const bool act = q < V.n_probes && active_state(step_state(V, ob, q));
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
// volume, volumes in order) and the frame's counters.
__global__ __launch_bounds__(kCompactBlock) void k_state_scatter(VolumeSet vs, CompactArgs A, FrameScratch fs) {
  __shared__ int wave_off[kCompactBlock / 64];
  __shared__ int s_base;
  __shared__ int s_slot[IRF_MAX_VOLUMES + 1];
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
  const uint8_t st = q < V.n_probes ? V.states[q] : (uint8_t)IRF_OFF;
  const bool act = active_state(st);
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
  if (act) write_slot(vs, fs, s_base + wave_off[wave] + __popcll(m & ((1ull << lane) - 1ull)), v, q, newly(st));
  if (b == 0 && threadIdx.x == 0) {
    int slot = 0;
    for (int u = 0; u < vs.n; u++) {
      s_slot[u] = slot;
      for (int i = A.block_base[u]; i < A.block_base[u + 1]; i++) slot += fs.block_active[i];
    }
    s_slot[vs.n] = slot;
    write_counters(vs, fs, s_slot);
  }
}

// ---- launches

FrameBegin make_frame_begin(const FrameParams& p, const VolumeSet& vs, ObjectBoxes ob, FrameScratch fs,
                            bool weights) {
  FrameBegin a;
  memset(&a, 0, sizeof(a));   // padding too: the struct is a captured node's argument
  a.p = p;
  a.vs = vs;
  a.ob = ob;
  a.fs = fs;
  int maxr = 0, P = 0;
  for (int v = 0; v < vs.n; v++) {
    maxr = vs.v[v].rays > maxr ? vs.v[v].rays : maxr;
    P += vs.v[v].n_probes;
  }
  a.dir_blocks = (maxr + kBeginBlock - 1) / kBeginBlock;
  a.row_waves = (maxr + 63) / 64 > 0 ? (maxr + 63) / 64 : 1;      // <= 16: at most 1024 rays
  const int rows_per_block = (kBeginBlock / 64) / a.row_waves;
  a.weight_rows = weights ? (kRows + rows_per_block - 1) / rows_per_block : 0;
  a.total_probes = P;
  a.compact = P <= kSmallProbes ? 1 : 0;
  return a;
}

void launch_frame_begin(const FrameBegin& a, hipStream_t s) {
  if (a.vs.n == 0) return;
  if (!a.compact) {
    CompactArgs A;
    A.block_base[0] = 0;
    for (int v = 0; v < a.vs.n; v++)
      A.block_base[v + 1] = A.block_base[v] + (a.vs.v[v].n_probes + kCompactBlock - 1) / kCompactBlock;
    irf_launch(k_state_count, dim3(A.block_base[a.vs.n]), dim3(kCompactBlock), 0, s, a.vs, a.ob, A, a.fs);
    irf_launch(k_state_scatter, dim3(A.block_base[a.vs.n]), dim3(kCompactBlock), 0, s, a.vs, A, a.fs);
  }
  irf_launch(k_frame_begin, dim3(a.dir_blocks + a.weight_rows + a.compact, a.vs.n), dim3(kBeginBlock), 0, s, a);
}

const void* frame_begin_kernel() { return (const void*)k_frame_begin; }

}  // namespace irf
