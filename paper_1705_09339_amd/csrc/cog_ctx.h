// Host-side definition of a stream context, shared by the one-stream calls
// (cog_api.cpp) and the batched tick (cog_batch.cpp).  Library-private.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "cog.h"
#include "cog_device.h"

namespace cog_rt {

// Statistics workspace: the per-tile rows of a launch (16 B per tile and
// frame) fill at most kRowBudget bytes, which sets the frames per launch
// when statistics are requested (between kChunkMin and kChunkMax); the
// reduced per-block sums of up to stat_frames frames collect on the device
// and are read back in one copy.
constexpr size_t kRowBudget = (size_t)32 << 20;
constexpr int kChunkMin = 16;
constexpr int kChunkMax = 64;
constexpr size_t kSumBudget = (size_t)8 << 20;
constexpr int kSumFramesMax = 4096;
// A cog_step_frames call with statistics over more frames than the chunk
// grows a row workspace of the context's own (kept until cog_destroy) so that
// up to kRowWorkspaceMax bytes of rows -- all its frames, usually -- go in one
// launch: every launch boundary costs a reload of the per-pixel state.
constexpr size_t kRowWorkspaceMax = (size_t)1 << 30;

// Device layout of one stream's state (all regions 256-byte aligned).
struct Plan {
  int64_t P = 0, Ppad = 0;
  int C = 0, K = 0, R = 0, RG = 0, PB = 0, sin = 1;
  int tile = 0, ppt = 1, ntiles = 0, nslots = 0, nblk = 0;
  bool auto_tile = false;  // tile_px = 0: the library picks the kernel per launch
  int stat_chunk = 0;      // frames per launch with statistics
  int stat_frames = 0;     // frames of reduced sums held on the device
  size_t off_gmm = 0, off_rga = 0, off_prior = 0, off_cnt = 0, off_sat = 0, off_gkey = 0,
         off_prev = 0, off_labels = 0, off_kdew = 0, off_partials = 0, off_statout = 0, total = 0;
};

cog_status fail(cog_ctx *h, cog_status s, const std::string &msg);
cog_status hip_fail(cog_ctx *h, hipError_t e, const char *what);

// Training of the pixels [p0, p1) on stream st (device frames; p0 a multiple
// of 128), and the context's switch to trained once every pixel has been
// trained: together they are cog_train_prior, which the serving loop issues
// in slices between its ticks.
cog_status train_range(cog_ctx *h, const void *dframes, int n, int64_t p0, int64_t p1,
                       hipStream_t st);
void train_finish(cog_ctx *h, int n);

// Per-frame statistics from the reduced counter blocks [n][nblk][kStat].
void fill_infos(const cog_ctx *h, int64_t first_frame, int n, const uint32_t *blocks,
                cog_step_info *infos, int nblk);

}  // namespace cog_rt

struct cog_ctx {
  cog_params p{};
  cog_rt::Plan plan;
  hipStream_t stream = nullptr;
  int device = 0;
  bool own_state = false;
  char *dstate = nullptr;
  cog::Buffers buf{};
  cog::KParams kp{};
  int32_t n_train = 0;
  int64_t frame = 0;
  void *stage_in = nullptr;
  size_t stage_in_cap = 0;
  uint8_t *stage_mask = nullptr;
  size_t stage_mask_cap = 0;
  std::vector<uint32_t> host_stats;
  std::string err;
  uint4 *rows_ws = nullptr;  // statistics rows of long calls (grown on demand)
  size_t rows_ws_bytes = 0;
  char *scratch = nullptr;  // this GPU's no-allocation grouping scratch (device address)
  std::string scratch_err;
};
