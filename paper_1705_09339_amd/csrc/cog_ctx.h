// Host-side definition of a stream context, shared by the one-stream calls
// (cog_api.cpp) and the batched tick (cog_batch.cpp).  Library-private.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "cog.h"
#include "cog_device.h"

namespace cog_rt {

constexpr int kChunk = 16;  // frames per launch when statistics are requested

// Device layout of one stream's state (all regions 256-byte aligned).
struct Plan {
  int64_t P = 0, Ppad = 0;
  int C = 0, K = 0, R = 0, RG = 0, PB = 0, sin = 1;
  int tile = 0, ppt = 1, ntiles = 0, nslots = 0, nblk = 0;
  size_t off_gmm = 0, off_rga = 0, off_prior = 0, off_cnt = 0, off_sat = 0, off_gkey = 0,
         off_prev = 0, off_labels = 0, off_kdew = 0, off_partials = 0, off_statout = 0, total = 0;
};

cog_status fail(cog_ctx *h, cog_status s, const std::string &msg);
cog_status hip_fail(cog_ctx *h, hipError_t e, const char *what);

// Per-frame statistics from the reduced counter blocks [n][nblk][kStat].
void fill_infos(const cog_ctx *h, int64_t first_frame, int n, const uint32_t *blocks,
                cog_step_info *infos);

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
  char *scratch = nullptr;  // this GPU's no-allocation grouping scratch (device address)
  std::string scratch_err;
};
