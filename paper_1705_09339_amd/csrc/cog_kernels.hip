// gfx950 kernels of the Cascade-of-Gaussians background subtractor
// (arXiv 1705.09339) that do not depend on the mixture size -- the per-frame
// statistics reduction and the spatio-temporal grouping -- and the launchers
// that dispatch the mixture-size templates (cog_kern.h, instantiated per K in
// cog_inst_k*.hip).
#include "cog_device.h"

#include <mutex>

namespace cog {
namespace {

// Statistics reduction: workgroup (blk, f) sums counters of slots
// [blk * kStatBlock, ...) of frame f.
__device__ __forceinline__ void stats_block(const StatJob &j, int blk, int f) {
  __shared__ uint32_t red[kNW][kStat];
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blk * kStatBlock;
  const int64_t s1 = s0 + kStatBlock < j.nslots ? s0 + kStatBlock : j.nslots;
  uint32_t acc[kStat];
#pragma unroll
  for (int k = 0; k < kStat; ++k) acc[k] = 0u;
  const uint4 *row = j.partials + (int64_t)f * j.nslots;
  for (int64_t i = s0 + tid; i < s1; i += kNT) {
    const uint4 a = row[i];
    acc[0] += a.x & 0xffffu; acc[1] += a.x >> 16;
    acc[2] += a.y & 0xffffu; acc[3] += a.y >> 16;
    acc[4] += a.z & 0xffffu; acc[5] += a.z >> 16;
    acc[6] += a.w;
  }
#pragma unroll
  for (int k = 0; k < kStat; ++k) {
    uint32_t v = acc[k];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
    acc[k] = v;
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int k = 0; k < kStat; ++k) red[tid >> 6][k] = acc[k];
  }
  __syncthreads();
  if (tid < kStat) {
    uint32_t v = 0u;
#pragma unroll
    for (int w = 0; w < kNW; ++w) v += red[w][tid];
    const int nblk = (j.nslots + kStatBlock - 1) / kStatBlock;
    j.out[((int64_t)f * nblk + blk) * kStat + tid] = v;
  }
}

__global__ __launch_bounds__(kNT) void k_stats(StatJob j) {
  if ((int)blockIdx.y >= j.nframes) return;
  if ((int64_t)blockIdx.x * kStatBlock >= j.nslots) return;
  stats_block(j, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kNT) void k_stats_table(const StatJob *jobs) {
  const StatJob j = jobs[blockIdx.z];
  if ((int)blockIdx.y >= j.nframes) return;
  if ((int64_t)blockIdx.x * kStatBlock >= j.nslots) return;
  stats_block(j, blockIdx.x, blockIdx.y);
}

// ============================================================================
// Spatio-temporal grouping (§2 "Clustering Similar Background"): integer
// k-means over the two warm-up keys of every pixel, then the one-sigma band
// of eq. 3.  One thread per pixel; per-block sums are exact integers, so
// the result does not depend on the order of the reduction.
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += (uint64_t)__shfl_xor((long long)v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  uint64_t t = 0;
#pragma unroll
  for (int i = 0; i < kNW; ++i) t += red[i];
  return t;
}

__global__ __launch_bounds__(kNT) void k_group_range(const uint2 *keys, int64_t P, uint64_t *part) {
  __shared__ uint64_t red[kNW];
  __shared__ uint32_t rlo[kNW], rhi[kNW];
  const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const bool valid = p < P;
  const uint2 k = valid ? keys[p] : make_uint2(0u, 0u);
  uint64_t out[6];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const uint32_t v = d ? k.y : k.x;
    // the wave's minimum and maximum by lane exchange, then the block's
    uint32_t lo = valid ? v : 0xffffffffu, hi = valid ? v : 0u;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const uint32_t l2 = (uint32_t)__shfl_xor((int)lo, o, 64), h2 = (uint32_t)__shfl_xor((int)hi, o, 64);
      lo = l2 < lo ? l2 : lo;
      hi = h2 > hi ? h2 : hi;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      rlo[threadIdx.x >> 6] = lo;
      rhi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    uint32_t blo = 0xffffffffu, bhi = 0u;
#pragma unroll
    for (int i = 0; i < kNW; ++i) {
      blo = rlo[i] < blo ? rlo[i] : blo;
      bhi = rhi[i] > bhi ? rhi[i] : bhi;
    }
    out[3 * d] = blo;
    out[3 * d + 1] = bhi;
    out[3 * d + 2] = block_sum_u64(valid ? (uint64_t)v : 0ull, red);
  }
  if (threadIdx.x < 6) part[(int64_t)blockIdx.x * 6 + threadIdx.x] = out[threadIdx.x];
}

__global__ __launch_bounds__(kNT) void k_group_assign(const uint2 *keys, int64_t P, GroupCenters c,
                                                      uint8_t *asg, uint64_t *part) {
  __shared__ uint64_t red[kNW];
  const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const bool valid = p < P;
  const uint2 k = valid ? keys[p] : make_uint2(0u, 0u);
  int best = 0;
  int64_t bd = 0;
#pragma unroll
  for (int g = 0; g < kGroups; ++g) {
    const int64_t a = (int64_t)k.x - c.c[g][0], b = (int64_t)k.y - c.c[g][1];
    const int64_t d = a * a + b * b;
    if (g == 0 || d < bd) {  // lowest index on ties
      bd = d;
      best = g;
    }
  }
  uint64_t changed = 0;
  if (valid) {
    changed = asg[p] != (uint8_t)best ? 1u : 0u;
    asg[p] = (uint8_t)best;
  }
  uint64_t out[kGroupStat];
  out[0] = block_sum_u64(changed, red);
#pragma unroll
  for (int g = 0; g < kGroups; ++g) {
    const bool in = valid && best == g;
    out[1 + 5 * g] = block_sum_u64(in ? 1ull : 0ull, red);
    out[2 + 5 * g] = block_sum_u64(in ? (uint64_t)k.x : 0ull, red);
    out[3 + 5 * g] = block_sum_u64(in ? (uint64_t)k.y : 0ull, red);
    out[4 + 5 * g] = block_sum_u64(in ? (uint64_t)k.x * k.x : 0ull, red);
    out[5 + 5 * g] = block_sum_u64(in ? (uint64_t)k.y * k.y : 0ull, red);
  }
  if (threadIdx.x < kGroupStat) part[(int64_t)blockIdx.x * kGroupStat + threadIdx.x] = out[threadIdx.x];
}

// The final map, and (cnt != nullptr) per-block counts of the grouped
// pixels of each cluster ([blocks][kGroups] u64).
__global__ __launch_bounds__(kNT) void k_group_map(const uint2 *keys, int64_t P, const uint8_t *asg,
                                                   GroupBands bands, uint8_t *map, uint64_t *cnt) {
  __shared__ uint64_t red[kNW];
  const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const bool valid = p < P;
  int g = 0;
  bool in = false;
  if (valid) {
    const uint2 k = keys[p];
    g = asg[p];
    in = true;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const double e = (double)(d ? k.y : k.x) - bands.mean[g][d];
      in = in && (fabs(e) <= bands.sd[g][d]);
    }
    map[p] = in ? (uint8_t)g : (uint8_t)255;
  }
  if (cnt) {  // uniform
    uint64_t out[kGroups];
#pragma unroll
    for (int q = 0; q < kGroups; ++q) out[q] = block_sum_u64(in && g == q ? 1ull : 0ull, red);
    if (threadIdx.x < kGroups) cnt[(int64_t)blockIdx.x * kGroups + threadIdx.x] = out[threadIdx.x];
  }
}

// Column reduction of per-block rows [nb][width] (width <= kGroupStat) into
// out[width] by one workgroup: field f is a minimum when bit f of minmask is
// set, a maximum for maxmask, else a sum.  Integer, so order-independent.
__global__ __launch_bounds__(kNT) void k_part_reduce(const uint64_t *part, int nb, int width,
                                                     uint32_t minmask, uint32_t maxmask,
                                                     uint64_t *out) {
  __shared__ uint64_t red[kNW][kGroupStat];
  uint64_t acc[kGroupStat];
#pragma unroll
  for (int f = 0; f < kGroupStat; ++f)
    acc[f] = ((minmask >> f) & 1u) ? ~0ull : 0ull;
  for (int i = threadIdx.x; i < nb; i += kNT) {
#pragma unroll
    for (int f = 0; f < kGroupStat; ++f) {
      if (f >= width) break;
      const uint64_t v = part[(int64_t)i * width + f];
      if ((minmask >> f) & 1u) acc[f] = v < acc[f] ? v : acc[f];
      else if ((maxmask >> f) & 1u) acc[f] = v > acc[f] ? v : acc[f];
      else acc[f] += v;
    }
  }
#pragma unroll
  for (int f = 0; f < kGroupStat; ++f) {
    uint64_t v = acc[f];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const uint64_t w = (uint64_t)__shfl_xor((long long)v, o, 64);
      if ((minmask >> f) & 1u) v = w < v ? w : v;
      else if ((maxmask >> f) & 1u) v = w > v ? w : v;
      else v += w;
    }
    acc[f] = v;
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int f = 0; f < kGroupStat; ++f) red[threadIdx.x >> 6][f] = acc[f];
  }
  __syncthreads();
  if (threadIdx.x < width) {
    const int f = threadIdx.x;
    uint64_t v = red[0][f];
    for (int w = 1; w < kNW; ++w) {
      const uint64_t x = red[w][f];
      if ((minmask >> f) & 1u) v = x < v ? x : v;
      else if ((maxmask >> f) & 1u) v = x > v ? x : v;
      else v += x;
    }
    out[f] = v;
  }
}

// One shared parameter set per group (§2 "Clustering Similar Background",
// the list's last item and eq. 3).  Per-block rows {count, sum} of each group
// and a flag of invalid input, [blocks][7] u64: a member's variance (the
// magnitude of the stored value) enters as rint(v * 2^16) in binary64, an
// exact integer below 2^53, so the sums are exact and order-independent.
__global__ __launch_bounds__(kNT) void k_share_sum(const float *rga, int rg, int c, int64_t P,
                                                   const uint8_t *map, uint64_t *part) {
  __shared__ uint64_t red[kNW];
  const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
  int g = 255;
  uint64_t q = 0, bad = 0;
  if (p < P) {
    g = map[p];
    if (g != 255) {
      const double v = rint((double)fabsf(rga[p * rg + c]) * 65536.0);
      if (g >= kGroups || !(v >= 0.0 && v < 9007199254740992.0)) bad = 1;
      else q = (uint64_t)v;
    }
  }
  uint64_t out[2 * kGroups + 1];
#pragma unroll
  for (int k = 0; k < kGroups; ++k) {
    const bool in = g == k && !bad;
    out[2 * k] = block_sum_u64(in ? 1ull : 0ull, red);
    out[2 * k + 1] = block_sum_u64(in ? q : 0ull, red);
  }
  out[2 * kGroups] = block_sum_u64(bad, red);
  if (threadIdx.x < 2 * kGroups + 1)
    part[(int64_t)blockIdx.x * (2 * kGroups + 1) + threadIdx.x] = out[threadIdx.x];
}

// Members take their group's shared variance, stored with the sign bit set
// (the cascade then uses it and never adapts it); every other pixel keeps the
// magnitude of its variance as its own (map == nullptr: every pixel).
__global__ __launch_bounds__(kNT) void k_share_set(float *rga, int rg, int c, int64_t P,
                                                   const uint8_t *map, ShareVars v) {
  const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (p >= P) return;
  const int g = map ? map[p] : 255;
  float *f = rga + p * rg + c;
  *f = g < kGroups ? __uint_as_float(__float_as_uint(v.var[g]) | 0x80000000u) : fabsf(*f);
}

__global__ __launch_bounds__(kNT) void k_fill_u8(uint8_t *p, int64_t n, uint8_t v) {
  for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kNT)
    p[i] = v;
}

// Scratch of the no-allocation grouping entry point: the assignment and map
// planes of up to kNoAllocMaxPixels pixels, the per-block rows and the
// reduced row.  One copy per GPU, held until the process ends.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

}  // namespace

#define COG_K_DISPATCH(CALL)      \
  switch (K) {                    \
    case 1: return CALL(1);       \
    case 2: return CALL(2);       \
    case 3: return CALL(3);       \
    case 4: return CALL(4);       \
    case 5: return CALL(5);       \
    case 6: return CALL(6);       \
    case 7: return CALL(7);       \
    case 8: return CALL(8);       \
    default: break;               \
  }

hipError_t launch_train(int C, int K, bool f32in, bool prior, bool aos, const Buffers &b,
                        const void *frames, int64_t stride, int n, const KParams &kp,
                        int64_t p0, int64_t p1, hipStream_t s) {
  if (prior != aos || p0 < 0 || p1 > b.P || (p0 & 127)) return hipErrorInvalidValue;
#define CALL(KK) launch_train_k<KK>(C, f32in, prior, b, frames, stride, n, kp, p0, p1, s)
  COG_K_DISPATCH(CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_cascade(int C, int K, bool f32in, int tile, const Buffers &b, const Frames &fr,
                          const KParams &kp, hipStream_t s) {
#define CALL(KK) launch_cascade_k<KK>(C, f32in, tile, b, fr, kp, s)
  COG_K_DISPATCH(CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_tick(int C, int K, bool f32in, bool lp, bool samp, TickHead *head,
                       const TickItem *items, int grid, int dynamic, hipStream_t s) {
#define CALL(KK) launch_tick_k<KK>(C, f32in, lp, samp, head, items, grid, dynamic, s)
  COG_K_DISPATCH(CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_tick_c(int C, int K, bool f32in, TickHead *head, const TickItem *items, int grid,
                         int dynamic, hipStream_t s) {
#define CALL(KK) launch_tick_c_k<KK>(C, f32in, head, items, grid, dynamic, s)
  COG_K_DISPATCH(CALL)
#undef CALL
  return hipErrorInvalidValue;
}

int tick_c_blocks_per_cu(int C, int K, bool f32in) {
#define CALL(KK) tick_c_blocks_per_cu_k<KK>(C, f32in)
  COG_K_DISPATCH(CALL)
#undef CALL
  return 0;
}

int tick_blocks_per_cu(int C, int K, bool f32in, bool lp, bool samp) {
#define CALL(KK) tick_blocks_per_cu_k<KK>(C, f32in, lp, samp)
  COG_K_DISPATCH(CALL)
#undef CALL
  return 0;
}

hipError_t launch_frame(int C, int K, bool f32in, const Buffers &b, const Frames &fr,
                        const KParams &kp, hipStream_t s) {
#define CALL(KK) launch_frame_k<KK>(C, f32in, b, fr, kp, s)
  COG_K_DISPATCH(CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_gmm(int C, int K, bool f32in, const Buffers &b, const Frames &fr,
                      const KParams &kp, hipStream_t s) {
#define CALL(KK) launch_gmm_k<KK>(C, f32in, b, fr, kp, s)
  COG_K_DISPATCH(CALL)
#undef CALL
  return hipErrorInvalidValue;
}

#undef COG_K_DISPATCH

int group_blocks(int64_t P) { return (int)((P + kNT - 1) / kNT); }

hipError_t launch_group_range(const uint2 *keys, int64_t P, uint64_t *part, hipStream_t s) {
  hipLaunchKernelGGL(k_group_range, dim3((unsigned)group_blocks(P)), dim3(kNT), 0, s, keys, P, part);
  return hipGetLastError();
}

hipError_t launch_group_assign(const uint2 *keys, int64_t P, const GroupCenters &c, uint8_t *asg,
                               uint64_t *part, hipStream_t s) {
  hipLaunchKernelGGL(k_group_assign, dim3((unsigned)group_blocks(P)), dim3(kNT), 0, s, keys, P, c,
                     asg, part);
  return hipGetLastError();
}

hipError_t launch_group_map(const uint2 *keys, int64_t P, const uint8_t *asg, const GroupBands &b,
                            uint8_t *map, uint64_t *cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_group_map, dim3((unsigned)group_blocks(P)), dim3(kNT), 0, s, keys, P, asg, b,
                     map, cnt);
  return hipGetLastError();
}

hipError_t launch_part_reduce(const uint64_t *part, int nb, int width, uint32_t minmask,
                              uint32_t maxmask, uint64_t *out, hipStream_t s) {
  if (width < 1 || width > kGroupStat || nb < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_part_reduce, dim3(1), dim3(kNT), 0, s, part, nb, width, minmask, maxmask, out);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + kNT - 1) / kNT;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)blocks), dim3(kNT), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_share_sum(const float *rga, int rg, int c, int64_t P, const uint8_t *map,
                            uint64_t *part, hipStream_t s) {
  hipLaunchKernelGGL(k_share_sum, dim3(group_blocks(P)), dim3(kNT), 0, s, rga, rg, c, P, map, part);
  return hipGetLastError();
}

hipError_t launch_share_set(float *rga, int rg, int c, int64_t P, const uint8_t *map,
                            const ShareVars &v, hipStream_t s) {
  hipLaunchKernelGGL(k_share_set, dim3(group_blocks(P)), dim3(kNT), 0, s, rga, rg, c, P, map, v);
  return hipGetLastError();
}

// The scratch's device address is looked up once per GPU, with that GPU
// current (every GPU holds its own copy at its own address), and kept; host
// code uses only these addresses, never the array's name.
hipError_t scratch_for_device(int device, char **out) {
  static std::mutex mu;
  static char *addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<char *>(ptr);
  }
  *out = addr[device];
  return hipSuccess;
}

hipError_t launch_stats(const StatJob &job, hipStream_t s) {
  if (job.nframes <= 0 || job.nslots <= 0) return hipSuccess;
  const unsigned nblk = (unsigned)((job.nslots + kStatBlock - 1) / kStatBlock);
  hipLaunchKernelGGL(k_stats, dim3(nblk, (unsigned)job.nframes, 1), dim3(kNT), 0, s, job);
  return hipGetLastError();
}

hipError_t launch_stats_table(const StatJob *jobs, int n, int max_blocks, int max_frames,
                              hipStream_t s) {
  if (n <= 0 || max_blocks <= 0 || max_frames <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stats_table, dim3((unsigned)max_blocks, (unsigned)max_frames, (unsigned)n),
                     dim3(kNT), 0, s, jobs);
  return hipGetLastError();
}

}  // namespace cog
