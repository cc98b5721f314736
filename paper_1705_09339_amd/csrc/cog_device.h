// Library-private declarations shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cog {

constexpr int kNT = 256;        // threads per workgroup (4 wave64)
constexpr int kNW = kNT / 64;   // waves per workgroup
constexpr int kBins = 16;       // prior bins per channel
constexpr int kStat = 8;        // reduced counters per block and frame:
                                // n0, n1, n2, n3, n3_bg, n_fg, n_skip, unused
// A kernel's statistics row per tile and frame: 16-bit counts packed in four
// words (a tile has at most 1024 pixels).
__host__ __device__ inline uint4 stat_row(uint32_t n0, uint32_t n1, uint32_t n2, uint32_t n3,
                                          uint32_t n3bg, uint32_t nfg, uint32_t nskip) {
  return make_uint4(n0 | (n1 << 16), n2 | (n3 << 16), n3bg | (nfg << 16), nskip);
}

// Floats of one pixel's mixture {w[K], var[K], mu[K][C]}.
__host__ __device__ constexpr int mix_floats(int C, int K) { return K * (C + 2); }
// Floats per per-pixel mixture record, padded to 16 B.  (Records padded to
// whole 128-byte lines were measured slower on the per-frame path: survivors
// cluster, so adjacent records share lines anyway, and the padding is read.)
__host__ __device__ constexpr int rec_floats(int C, int K) { return (mix_floats(C, K) + 3) & ~3; }
// Floats per running-average record {mu_r[C], var_r}.
__host__ __device__ constexpr int rga_floats(int C) { return C == 3 ? 4 : 2; }
// Bytes per prior record {t[C][16] u8, a, b, g f32} padded to 32/64 B.
__host__ __device__ constexpr int prior_bytes(int C) { return C == 3 ? 64 : 32; }

// Scalar parameters as the kernels use them (squares and complements
// rounded once to binary32 on the host).
struct KParams {
  float alpha, T, lam2, var_init, var_min;
  float tau_fd, lam_r2, alpha_rga, one_m_alpha_rga;
  float res_e1, res_e2, lam_m2, conf_thr, p_null, kappa;
  float nm1;            // n_train - 1
  float in_lo, q_scale; // f32 input quantisation: floor((v - in_lo) * q_scale)
  uint32_t stage_mask;
  uint32_t samp_window, samp_period;  // sampling: saturation window, evaluation period
  float lam_s2;                       // sampling: confidence gate squared
  float inv_res_e2;  // 1 / res_e2 correctly rounded when res_e2 is in [2^-20, 2^20], else 0
};

// Device state of one stream (see the host planner for sizes).
struct Buffers {
  float *gmm;                  // cascade: AoS records; baseline: 64-pixel AoSoA groups
  float *rga;                  // rga_floats(C) per pixel
  uint8_t *prior;              // prior_bytes(C) per pixel
  uint16_t *cnt;               // residue counts, 4 u16 per pixel (export only)
  void *prev;                  // C values per pixel (u8 or f32, as the input)
  unsigned long long *labels;  // 1 bit per pixel, bit p&63 of word p>>6
  const uint16_t *kdew;        // prior kernel weights, level-major [256][16]
  uint16_t *sat;               // sampling: consecutive confident frames per pixel
  uint2 *gkey;                 // grouping keys of the training warm-up, per pixel
  int64_t P;
};

// A run of consecutive frames handed to one launch.
struct Frames {
  const void *x;       // frame 0 (HWC)
  int64_t stride;      // elements between frames
  uint8_t *mask;       // mask of frame 0 or nullptr
  int64_t mstride;     // bytes between masks
  uint4 *partials;     // statistics rows [nframes][nslots] (stat_row) or nullptr
  int nslots;
  int nframes;
  int64_t frame0;      // index of frame 0 in the stream (sampling phase)
};

// ---- batched tick ------------------------------------------------------------
// One stream's work in a tick: its frames, state and parameters.  The tick's
// 64-pixel tiles are numbered consecutively over its items in item order;
// item i owns tiles [tile_begin, tile_begin + ceil(P / 64)).
struct TickItem {
  Frames fr;
  Buffers b;
  KParams kp;
  int32_t pad;
  int64_t tile_begin;
};

// Head of one class's work list.  queue is the dynamic schedule's next unit
// and must be zero when the launch starts (the host uploads it as zero).
struct TickHead {
  int64_t total_tiles;
  int32_t n_items;
  int32_t group;     // tiles per schedule unit
  uint32_t queue;
  uint32_t pad[11];
};

// Per-frame reduction of the per-tile counters of one run of frames:
// out[f][blk][kStat] = sums over the slots of block blk (kStatBlock slots).
struct StatJob {
  const uint4 *partials;     // rows [nframes][nslots]
  uint32_t *out;             // [nframes][ceil(nslots / kStatBlock)][kStat]
  int32_t nslots;
  int32_t nframes;
};
constexpr int kStatBlock = 4096;

// ---- spatio-temporal grouping --------------------------------------------------
constexpr int kGroups = 3;
// Per-block sums of one assignment pass: changed, then per group count,
// key sums (2) and key square sums (2).
constexpr int kGroupStat = 1 + kGroups * 5;
struct GroupCenters {
  int64_t c[kGroups][2];
};
struct GroupBands {
  double mean[kGroups][2], sd[kGroups][2];
};

// Launchers (cog_kernels.hip).  Return hipSuccess or the launch error.
// Training of the pixels [p0, p1) (the frames hold every pixel; slices of a
// stream start at multiples of 128 pixels, so each label word is written by
// one launch).
hipError_t launch_train(int C, int K, bool f32in, bool prior, bool aos, const Buffers &b,
                        const void *frames, int64_t stride, int n, const KParams &kp,
                        int64_t p0, int64_t p1, hipStream_t s);
hipError_t launch_cascade(int C, int K, bool f32in, int tile, const Buffers &b, const Frames &fr,
                          const KParams &kp, hipStream_t s);
hipError_t launch_gmm(int C, int K, bool f32in, const Buffers &b, const Frames &fr,
                      const KParams &kp, hipStream_t s);
// One frame (fr.nframes == 1, no sampling) in 256-pixel tiles with compacted
// survivors; its statistics rows have ceil(P / kFrameTile) slots.
#ifndef COG_FRAME_TILE
#define COG_FRAME_TILE 256
#endif
constexpr int kFrameTile = COG_FRAME_TILE;
hipError_t launch_frame(int C, int K, bool f32in, const Buffers &b, const Frames &fr,
                        const KParams &kp, hipStream_t s);
// Persistent tick over one class (C, K, input type) of streams: grid
// workgroups of one wave; dynamic = 0 deals units round-robin by workgroup,
// 1 hands them out from head->queue.
hipError_t launch_tick(int C, int K, bool f32in, bool lp, bool samp, TickHead *head,
                       const TickItem *items, int grid, int dynamic, hipStream_t s);
// The compacting tick: every item advances by one frame (no sampling) in
// kFrameTile-pixel tiles; item i owns tiles [tile_begin, + ceil(P / kFrameTile)).
hipError_t launch_tick_c(int C, int K, bool f32in, TickHead *head, const TickItem *items, int grid,
                         int dynamic, hipStream_t s);
int tick_c_blocks_per_cu(int C, int K, bool f32in);
// Statistics reduction: one job by value, or n jobs from a device table
// (grid covers max_blocks x max_frames x n).
hipError_t launch_stats(const StatJob &job, hipStream_t s);
hipError_t launch_stats_table(const StatJob *jobs, int n, int max_blocks, int max_frames,
                              hipStream_t s);
// Grouping: per-block {min, max, sum} of both keys ([blocks][6] u64), one
// assignment pass (asg in/out, [blocks][kGroupStat] u64), and the final map.
int group_blocks(int64_t P);
// One shared variance per group: per-block rows {count, sum} x 3 and an
// invalid-input count ([blocks][7] u64, reduced with launch_part_reduce),
// then the stores of the members' shared variances (sign bit set) and of
// the other pixels' own (map == nullptr: every pixel ungrouped).
struct ShareVars {
  float var[kGroups];
};
hipError_t launch_share_sum(const float *rga, int rg, int c, int64_t P, const uint8_t *map,
                            uint64_t *part, hipStream_t s);
hipError_t launch_share_set(float *rga, int rg, int c, int64_t P, const uint8_t *map,
                            const ShareVars &v, hipStream_t s);
hipError_t launch_group_range(const uint2 *keys, int64_t P, uint64_t *part, hipStream_t s);
hipError_t launch_group_assign(const uint2 *keys, int64_t P, const GroupCenters &c, uint8_t *asg,
                               uint64_t *part, hipStream_t s);
hipError_t launch_group_map(const uint2 *keys, int64_t P, const uint8_t *asg, const GroupBands &b,
                            uint8_t *map, uint64_t *cnt, hipStream_t s);
// out[f] = column f of part[nb][width] reduced by minimum (bit f of minmask),
// maximum (maxmask) or sum; one workgroup.
hipError_t launch_part_reduce(const uint64_t *part, int nb, int width, uint32_t minmask,
                              uint32_t maxmask, uint64_t *out, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s);

// Static scratch of the no-allocation grouping call: the assignment plane,
// the map plane, per-block rows, the reduced row.
constexpr int64_t kNoAllocMaxPixels = (int64_t)1 << 23;  // 8 Mpx: 3840 x 2160 fits
constexpr size_t kScratchAsg = 0;
constexpr size_t kScratchMap = (size_t)kNoAllocMaxPixels;
constexpr size_t kScratchPart = 2 * (size_t)kNoAllocMaxPixels;
constexpr size_t kScratchRed =
    kScratchPart + (size_t)(kNoAllocMaxPixels / kNT) * kGroupStat * sizeof(uint64_t);
constexpr size_t kNoAllocScratchBytes = kScratchRed + 256;
// Device address of GPU `device`'s copy of the scratch; the first call for a
// GPU must have that GPU current.
constexpr int kMaxDevices = 64;
hipError_t scratch_for_device(int device, char **out);
// Workgroups of the class's tick kernel one compute unit keeps resident
// (0 if the query fails).
int tick_blocks_per_cu(int C, int K, bool f32in, bool lp, bool samp);

// The same launchers for one mixture size K (cog_kern.h), instantiated for
// K = 1..8, one translation unit each; the calls above dispatch on K.
template <int K>
hipError_t launch_train_k(int C, bool f32in, bool prior, const Buffers &b, const void *frames,
                          int64_t stride, int n, const KParams &kp, int64_t p0, int64_t p1,
                          hipStream_t s);
template <int K>
hipError_t launch_cascade_k(int C, bool f32in, int tile, const Buffers &b, const Frames &fr,
                            const KParams &kp, hipStream_t s);
template <int K>
hipError_t launch_tick_k(int C, bool f32in, bool lp, bool samp, TickHead *head,
                         const TickItem *items, int grid, int dynamic, hipStream_t s);
template <int K>
int tick_blocks_per_cu_k(int C, bool f32in, bool lp, bool samp);
template <int K>
hipError_t launch_tick_c_k(int C, bool f32in, TickHead *head, const TickItem *items, int grid,
                           int dynamic, hipStream_t s);
template <int K>
int tick_c_blocks_per_cu_k(int C, bool f32in);
template <int K>
hipError_t launch_frame_k(int C, bool f32in, const Buffers &b, const Frames &fr, const KParams &kp,
                          hipStream_t s);
template <int K>
hipError_t launch_gmm_k(int C, bool f32in, const Buffers &b, const Frames &fr, const KParams &kp,
                        hipStream_t s);

}  // namespace cog
