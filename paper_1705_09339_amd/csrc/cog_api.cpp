// Host runtime of the C ABI declared in include/cog.h.
#include "cog.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cog_ctx.h"
#include "cog_device.h"

namespace {

thread_local std::string g_err;

constexpr uint32_t kMagic = 0x31474F43u;  // "COG1"
using cog_rt::Plan;

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }
size_t pad64(size_t n) { return (n + 63) & ~(size_t)63; }

}  // namespace

namespace cog_rt {

cog_status fail(cog_ctx *h, cog_status s, const std::string &msg) {
  if (h) h->err = msg;
  g_err = msg;
  return s;
}

cog_status hip_fail(cog_ctx *h, hipError_t e, const char *what) {
  return fail(h, COG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void fill_infos(const cog_ctx *h, int64_t first_frame, int n, const uint32_t *blocks,
                cog_step_info *infos, int nb) {
  for (int f = 0; f < n; ++f) {
    int64_t s[cog::kStat] = {0, 0, 0, 0, 0, 0, 0, 0};
    const uint32_t *row = blocks + (size_t)f * nb * cog::kStat;
    for (int i = 0; i < nb; ++i)
      for (int k = 0; k < cog::kStat; ++k) s[k] += row[(size_t)i * cog::kStat + k];
    cog_step_info &o = infos[f];
    o.frame = first_frame + f;
    for (int k = 0; k < 4; ++k) o.n_stage[k] = s[k];
    o.n3_bg = s[4];
    o.n_fg = s[5];
    o.illum_flag = ((double)s[3] > (double)h->p.illum_frac * (double)h->plan.P) ? 1 : 0;
    o.n_skip = (int32_t)s[6];
  }
}

}  // namespace cog_rt

using cog_rt::fail;
using cog_rt::hip_fail;

namespace {

// Validation of the parameter block; returns an empty string when valid.
std::string check_params(const cog_params *p) {
  if (!p) return "params is NULL";
  if (p->struct_size != sizeof(cog_params)) return "params.struct_size mismatch";
  if (p->width <= 0 || p->height <= 0) return "width and height must be positive";
  if ((int64_t)p->width * p->height > ((int64_t)1 << 28)) return "frame too large (at most 2^28 pixels)";
  if (p->channels != 1 && p->channels != 3) return "channels must be 1 or 3";
  if (p->dtype != COG_U8 && p->dtype != COG_F32) return "dtype must be COG_U8 or COG_F32";
  if (p->dtype == COG_F32 && !(p->in_hi > p->in_lo)) return "in_hi must exceed in_lo";
  if (p->K < 1 || p->K > 8) return "K must be in [1, 8]";
  if (!(p->alpha > 0.0f && p->alpha <= 1.0f)) return "alpha must be in (0, 1]";
  if (!(p->T > 0.0f && p->T <= 1.0f)) return "T must be in (0, 1]";
  if (!(p->lambda > 0.0f)) return "lambda must be positive";
  if (!(p->var_min > 0.0f) || !(p->var_init >= p->var_min)) return "need 0 < var_min <= var_init";
  if (p->stage_mask & ~15u) return "unknown stage_mask bits";
  if (p->stage_mask & COG_STAGE_SAMPLE) {
    if (p->path != COG_PATH_CASCADE) return "sampling is a cascade option";
    if (p->samp_window < 1 || p->samp_window > 65535) return "samp_window must be in [1, 65535]";
    if (p->samp_period < 1 || p->samp_period > 65535) return "samp_period must be in [1, 65535]";
    if (!(p->samp_lambda >= 0.0f)) return "samp_lambda must be >= 0";
  }
  if (!(p->tau_fd >= 0.0f)) return "tau_fd must be >= 0";
  if (!(p->lambda_rga >= 0.0f)) return "lambda_rga must be >= 0";
  if (!(p->alpha_rga > 0.0f && p->alpha_rga <= 1.0f)) return "alpha_rga must be in (0, 1]";
  if (p->kde_bins != 16) return "kde_bins must be 16";
  if (!(p->kde_h > 0.0f)) return "kde_h must be positive";
  if (!(p->res_e2 > 0.0f) || !(p->res_e1 <= p->res_e2)) return "need res_e1 <= res_e2, res_e2 > 0";
  if (!(p->lambda_m > 0.0f)) return "lambda_m must be positive";
  if (!(p->kappa_alpha >= 0.0f && p->kappa_alpha <= 1.0f)) return "kappa_alpha must be in [0, 1]";
  if (!(p->illum_frac >= 0.0f)) return "illum_frac must be >= 0";
  if (p->path != COG_PATH_CASCADE && p->path != COG_PATH_GMM) return "unknown path";
  if (p->tile_px != 0 && p->tile_px != 64 && p->tile_px != 128 && p->tile_px != 256 &&
      p->tile_px != 512 && p->tile_px != 1024)
    return "tile_px must be 0, 64, 128, 256, 512 or 1024";
  return std::string();
}

Plan make_plan(const cog_params *p) {
  Plan pl;
  pl.P = (int64_t)p->width * p->height;
  pl.Ppad = (pl.P + 63) & ~(int64_t)63;
  pl.C = p->channels;
  pl.K = p->K;
  pl.R = cog::rec_floats(pl.C, pl.K);
  pl.RG = cog::rga_floats(pl.C);
  pl.PB = cog::prior_bytes(pl.C);
  pl.sin = p->dtype == COG_U8 ? 1 : 4;
  const bool cascade = p->path == COG_PATH_CASCADE;
  if (cascade) {
    int tile = p->tile_px;
    pl.auto_tile = tile == 0;
    if (tile == 0) tile = 64;
    pl.tile = tile;
    pl.ppt = tile >= cog::kNT ? tile / cog::kNT : tile / 64;
    pl.ntiles = (int)((pl.P + tile - 1) / tile);
    pl.nslots = pl.ntiles;
  } else {
    pl.tile = 64;
    pl.ppt = 1;
    pl.ntiles = (int)((pl.P + 63) / 64);
    pl.nslots = pl.ntiles;
  }
  size_t off = 0;
  pl.off_gmm = off;
  off += align256((size_t)pl.Ppad * pl.R * 4);
  pl.off_rga = off;
  if (cascade) off += align256((size_t)pl.Ppad * pl.RG * 4);
  pl.off_prior = off;
  if (cascade) off += align256((size_t)pl.Ppad * pl.PB);
  pl.off_cnt = off;
  if (cascade) off += align256((size_t)pl.Ppad * 8);
  pl.off_sat = off;
  if (cascade) off += align256((size_t)pl.Ppad * 2);
  pl.off_gkey = off;
  if (cascade) off += align256((size_t)pl.Ppad * 8);
  pl.off_prev = off;
  off += align256((size_t)pl.Ppad * pl.C * pl.sin);
  pl.off_labels = off;
  off += align256((size_t)(pl.Ppad / 64) * 8);
  pl.off_kdew = off;
  off += align256(256 * 16 * 2);
  pl.off_partials = off;
  const size_t row_bytes = (size_t)pl.nslots * 16;
  pl.stat_chunk = (int)std::max<size_t>(cog_rt::kChunkMin,
                                        std::min<size_t>(cog_rt::kChunkMax, cog_rt::kRowBudget / row_bytes));
  off += align256((size_t)pl.stat_chunk * row_bytes);
  pl.nblk = (pl.nslots + cog::kStatBlock - 1) / cog::kStatBlock;
  const size_t sum_bytes = (size_t)pl.nblk * cog::kStat * 4;
  pl.stat_frames = (int)std::max<size_t>((size_t)pl.stat_chunk,
                                         std::min<size_t>(cog_rt::kSumFramesMax, cog_rt::kSumBudget / sum_bytes));
  pl.off_statout = off;
  off += align256((size_t)pl.stat_frames * sum_bytes);
  pl.total = off;
  return pl;
}

// W[b][v] = rint(65535 * sum_{u in bin b} phi(u - v)), phi the Gaussian
// kernel of bandwidth h normalised over [-1024, 1024]; row-major [16][256].
void kde_table(double h, uint16_t *out) {
  const double den = 2.0 * h * h;
  double z = 0.0;
  for (int e = -1024; e <= 1024; ++e) z += std::exp(-(double)(e * e) / den);
  for (int b = 0; b < 16; ++b) {
    for (int v = 0; v < 256; ++v) {
      double s = 0.0;
      for (int u = 16 * b; u < 16 * b + 16; ++u) {
        const int d = u - v;
        s += std::exp(-(double)(d * d) / den) / z;
      }
      out[b * 256 + v] = (uint16_t)std::rint(65535.0 * s);
    }
  }
}

cog::KParams make_kparams(const cog_params *p, int32_t n_train) {
  cog::KParams k{};
  k.alpha = p->alpha;
  k.T = p->T;
  k.lam2 = p->lambda * p->lambda;
  k.var_init = p->var_init;
  k.var_min = p->var_min;
  k.tau_fd = p->tau_fd;
  k.lam_r2 = p->lambda_rga * p->lambda_rga;
  k.alpha_rga = p->alpha_rga;
  k.one_m_alpha_rga = 1.0f - p->alpha_rga;
  k.res_e1 = p->res_e1;
  k.res_e2 = p->res_e2;
  k.lam_m2 = p->lambda_m * p->lambda_m;
  k.conf_thr = p->conf_thr;
  k.p_null = p->p_null;
  k.kappa = p->kappa_alpha;
  k.nm1 = (float)(n_train - 1);
  k.in_lo = p->in_lo;
  k.q_scale = 256.0f / (p->in_hi - p->in_lo);
  k.stage_mask = p->stage_mask;
  k.samp_window = (uint32_t)(p->samp_window > 0 ? p->samp_window : 1);
  k.samp_period = (uint32_t)(p->samp_period > 0 ? p->samp_period : 1);
  k.lam_s2 = p->samp_lambda * p->samp_lambda;
  // the cascade divides integer frame differences by res_e2 through this
  // reciprocal (exact in that range; outside it, it divides)
  k.inv_res_e2 = (p->res_e2 >= 0x1p-20f && p->res_e2 <= 0x1p20f) ? 1.0f / p->res_e2 : 0.0f;
  return k;
}

cog_status ensure_stage(cog_ctx *h, size_t in_bytes, size_t mask_bytes) {
  if (in_bytes > h->stage_in_cap) {
    if (h->stage_in) (void)hipFree(h->stage_in);
    h->stage_in = nullptr;
    h->stage_in_cap = 0;
    hipError_t e = hipMalloc(&h->stage_in, in_bytes);
    if (e != hipSuccess) return fail(h, COG_E_OOM, "staging allocation failed");
    h->stage_in_cap = in_bytes;
  }
  if (mask_bytes > h->stage_mask_cap) {
    if (h->stage_mask) (void)hipFree(h->stage_mask);
    h->stage_mask = nullptr;
    h->stage_mask_cap = 0;
    hipError_t e = hipMalloc((void **)&h->stage_mask, mask_bytes);
    if (e != hipSuccess) return fail(h, COG_E_OOM, "staging allocation failed");
    h->stage_mask_cap = mask_bytes;
  }
  return COG_OK;
}

// Runs n frames starting at frames (device) writing masks (device or NULL).
// With statistics the frames go in launches of at most stat_chunk frames;
// each launch's rows are reduced on the device into the sums buffer, which
// is read back (one copy, one synchronisation) when full and at the end.
cog_status run_frames(cog_ctx *h, const void *dframes, int n, uint8_t *dmasks, bool want_stats,
                      cog_step_info *infos) {
  const Plan &pl = h->plan;
  const int64_t fstride = pl.P * pl.C;  // elements
  const size_t esz = (size_t)pl.sin;
  uint32_t *sums = reinterpret_cast<uint32_t *>(h->dstate + pl.off_statout);
  const size_t sum_cap = (size_t)pl.stat_frames * pl.nblk * cog::kStat;  // words
  struct Pending { int first, cnt, nblk; size_t off; };
  std::vector<Pending> pend;
  size_t used = 0;
  auto flush = [&]() -> cog_status {
    if (pend.empty()) return COG_OK;
    h->host_stats.resize(used);
    hipError_t e = hipMemcpyAsync(h->host_stats.data(), sums, used * 4, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "statistics copy");
    for (const Pending &q : pend)
      cog_rt::fill_infos(h, h->frame + q.first, q.cnt, h->host_stats.data() + q.off, infos + q.first,
                         q.nblk);
    pend.clear();
    used = 0;
    return COG_OK;
  };
  // rows of the launches: the state's chunk, or the grown workspace
  uint4 *rows = reinterpret_cast<uint4 *>(h->dstate + pl.off_partials);
  int chunk = pl.stat_chunk;
  if (want_stats && n > pl.stat_chunk) {
    const size_t row_bytes = (size_t)pl.nslots * 16;
    const size_t want = std::min((size_t)n * row_bytes, cog_rt::kRowWorkspaceMax / row_bytes * row_bytes);
    if (want > h->rows_ws_bytes) {
      uint4 *p = nullptr;
      if (hipMalloc((void **)&p, want) == hipSuccess) {
        if (h->rows_ws) {
          (void)hipStreamSynchronize(h->stream);  // earlier launches may still read the old rows
          (void)hipFree(h->rows_ws);
        }
        h->rows_ws = p;
        h->rows_ws_bytes = want;
      } else {
        (void)hipGetLastError();  // keep the smaller workspace (or the chunk)
      }
    }
    if (h->rows_ws && h->rows_ws_bytes / row_bytes > (size_t)chunk) {
      rows = h->rows_ws;
      // (a launch's sums must fit the device sums buffer too)
      chunk = (int)std::min<size_t>(std::min<size_t>(h->rows_ws_bytes / row_bytes, (size_t)n),
                                    (size_t)pl.stat_frames);
    }
  }
  int done = 0;
  while (done < n) {
    const int cnt = want_stats ? std::min(chunk, n - done) : (n - done);
    cog::Frames fr{};
    fr.x = static_cast<const char *>(dframes) + (size_t)done * fstride * esz;
    fr.stride = fstride;
    fr.mask = dmasks ? dmasks + (size_t)done * pl.P : nullptr;
    fr.mstride = pl.P;
    fr.partials = want_stats ? rows : nullptr;
    fr.nframes = cnt;
    fr.frame0 = h->frame + done;
    // one frame with the automatic tile choice: the per-frame kernel, whose
    // 256-pixel tiles compact the survivors (the multi-frame kernel keeps the
    // dense state in registers across frames instead)
    const bool cascade = h->p.path == COG_PATH_CASCADE;
    const bool one = cascade && pl.auto_tile && cnt == 1 && !(h->p.stage_mask & COG_STAGE_SAMPLE);
    const int nslots = one ? (int)((pl.P + cog::kFrameTile - 1) / cog::kFrameTile) : pl.nslots;
    fr.nslots = nslots;
    hipError_t e;
    if (one)
      e = cog::launch_frame(pl.C, pl.K, h->p.dtype == COG_F32, h->buf, fr, h->kp, h->stream);
    else if (cascade)
      e = cog::launch_cascade(pl.C, pl.K, h->p.dtype == COG_F32, pl.tile, h->buf, fr, h->kp,
                              h->stream);
    else
      e = cog::launch_gmm(pl.C, pl.K, h->p.dtype == COG_F32, h->buf, fr, h->kp, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "kernel launch");
    if (want_stats) {
      // per-frame sums of this launch on the device, beside the earlier ones
      const int nblk = (nslots + cog::kStatBlock - 1) / cog::kStatBlock;
      const size_t nw = (size_t)cnt * nblk * cog::kStat;
      if (used + nw > sum_cap) {
        cog_status s = flush();
        if (s != COG_OK) return s;
      }
      cog::StatJob job{};
      job.partials = fr.partials;
      job.out = sums + used;
      job.nslots = nslots;
      job.nframes = cnt;
      e = cog::launch_stats(job, h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "statistics launch");
      pend.push_back(Pending{done, cnt, nblk, used});
      used += nw;
    }
    done += cnt;
  }
  return flush();
}

// Grouping preconditions shared by both entry points.
cog_status group_check(cog_ctx *h) {
  if (!h) return fail(nullptr, COG_E_INVALID, "context is NULL");
  if (h->p.path != COG_PATH_CASCADE) return fail(h, COG_E_UNSUPPORTED, "grouping needs the cascade path");
  if (h->n_train == 0) return fail(h, COG_E_STATE, "cog_train_prior has not run");
  return COG_OK;
}

// The grouping on caller-provided device scratch: asg and smap P bytes each
// (smap used when map_out is not a device buffer), part group_blocks(P) *
// kGroupStat words, red kGroupStat words.  Every per-block row is reduced on
// the device, so the host reads a few words per pass into its stack.
cog_status group_run(cog_ctx *h, uint8_t *map_out, int32_t map_on_device, cog_group_info *info,
                     uint8_t *asg, uint8_t *smap, uint64_t *part, uint64_t *red) {
  const int64_t P = h->plan.P;
  const int nb = cog::group_blocks(P);
  const uint2 *keys = h->buf.gkey;
  hipStream_t st = h->stream;
  cog_status rc = COG_OK;
  uint64_t row[cog::kGroupStat];
  auto check = [&](hipError_t e, const char *what) {
    if (e != hipSuccess && rc == COG_OK) rc = hip_fail(h, e, what);
    return rc == COG_OK;
  };
  auto reduce = [&](int width, uint32_t minmask, uint32_t maxmask) {
    return check(cog::launch_part_reduce(part, nb, width, minmask, maxmask, red, st), "grouping launch") &&
           check(hipMemcpyAsync(row, red, (size_t)width * 8, hipMemcpyDeviceToHost, st), "copy") &&
           check(hipStreamSynchronize(st), "grouping");
  };
  uint8_t *dmap = map_out && map_on_device ? map_out : smap;
  cog::GroupCenters c{};
  cog::GroupBands bands{};
  int it = 0;
  uint64_t cnt[cog::kGroups] = {0}, s1[cog::kGroups][2] = {{0}}, s2[cog::kGroups][2] = {{0}};
  // initial centres: minimum, floor of the mean, maximum of each key
  // (per-block rows {min, max, sum} for each key)
  if (check(cog::launch_group_range(keys, P, part, st), "grouping launch") &&
      reduce(6, 0x9u, 0x12u)) {
    for (int d = 0; d < 2; ++d) {
      c.c[0][d] = (int64_t)row[3 * d];
      c.c[1][d] = (int64_t)(row[3 * d + 2] / (uint64_t)P);
      c.c[2][d] = (int64_t)row[3 * d + 1];
    }
  }
  if (rc == COG_OK) check(cog::launch_fill_u8(asg, P, 255, st), "grouping launch");
  // Lloyd passes until no assignment changes
  for (it = 1; rc == COG_OK && it <= 32; ++it) {
    if (!check(cog::launch_group_assign(keys, P, c, asg, part, st), "grouping launch") ||
        !reduce(cog::kGroupStat, 0u, 0u))
      break;
    const uint64_t changed = row[0];
    for (int g = 0; g < cog::kGroups; ++g) {
      cnt[g] = row[1 + 5 * g];
      s1[g][0] = row[2 + 5 * g];
      s1[g][1] = row[3 + 5 * g];
      s2[g][0] = row[4 + 5 * g];
      s2[g][1] = row[5 + 5 * g];
    }
    if (changed == 0) break;
    for (int g = 0; g < cog::kGroups; ++g)
      if (cnt[g])
        for (int d = 0; d < 2; ++d) c.c[g][d] = (int64_t)(s1[g][d] / cnt[g]);
  }
  if (it > 32) it = 32;
  // eq. 3: one standard deviation around each cluster's member mean
  for (int g = 0; g < cog::kGroups; ++g)
    for (int d = 0; d < 2; ++d) {
      if (!cnt[g]) {
        bands.mean[g][d] = bands.sd[g][d] = 0.0;
        continue;
      }
      const double n = (double)cnt[g];
      bands.mean[g][d] = (double)s1[g][d] / n;
      const double var = (double)s2[g][d] / n - bands.mean[g][d] * bands.mean[g][d];
      bands.sd[g][d] = var > 0.0 ? std::sqrt(var) : 0.0;
    }
  if (rc == COG_OK)
    check(cog::launch_group_map(keys, P, asg, bands, dmap, info ? part : nullptr, st),
          "grouping launch");
  if (rc == COG_OK && info) reduce(cog::kGroups, 0u, 0u);
  if (rc == COG_OK && map_out && !map_on_device)
    check(hipMemcpyAsync(map_out, dmap, (size_t)P, hipMemcpyDeviceToHost, st), "copy");
  if (rc == COG_OK) check(hipStreamSynchronize(st), "grouping");
  if (rc == COG_OK && info) {
    std::memset(info, 0, sizeof(*info));
    info->iterations = it;
    for (int g = 0; g < cog::kGroups; ++g) {
      cog_group_stats &o = info->group[g];
      o.count = (int64_t)cnt[g];
      o.grouped = (int64_t)row[g];
      for (int d = 0; d < 2; ++d) {
        o.center[d] = c.c[g][d];
        o.mean[d] = bands.mean[g][d];
        o.sd[d] = bands.sd[g][d];
      }
    }
  }
  return rc;
}

}  // namespace

extern "C" {

cog_status cog_default_params(cog_params *p, int32_t w, int32_t h, int32_t c, int32_t dtype,
                              int32_t K) {
  if (!p) return fail(nullptr, COG_E_INVALID, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(cog_params);
  p->width = w;
  p->height = h;
  p->channels = c;
  p->dtype = dtype;
  p->in_lo = 0.0f;
  p->in_hi = 256.0f;
  p->K = K;
  p->alpha = 0.01f;
  p->T = 0.7f;
  p->lambda = 2.5f;
  p->var_init = (float)c * 225.0f;
  p->var_min = (float)c * 4.0f;
  p->stage_mask = COG_STAGE_ALL;
  p->tau_fd = 0.0f;
  p->lambda_rga = 2.5f;
  p->alpha_rga = p->alpha;
  p->kde_bins = 16;
  p->kde_h = 8.0f;
  p->res_e1 = 16.0f;
  p->res_e2 = 48.0f;
  p->lambda_m = 2.0f * p->lambda_rga;
  p->conf_thr = 0.5f;
  p->p_null = 0.1f;
  p->kappa_alpha = 0.5f;
  p->illum_frac = 0.7f;
  p->path = COG_PATH_CASCADE;
  p->tile_px = 0;
  p->samp_window = 32;
  p->samp_period = 4;
  p->samp_lambda = p->lambda_rga;
  return COG_OK;
}

cog_status cog_state_bytes(const cog_params *p, size_t *bytes) {
  const std::string e = check_params(p);
  if (!e.empty()) return fail(nullptr, COG_E_INVALID, e);
  if (!bytes) return fail(nullptr, COG_E_INVALID, "bytes is NULL");
  *bytes = make_plan(p).total;
  return COG_OK;
}

cog_status cog_canonical_bytes(const cog_params *p, size_t *bytes) {
  const std::string e = check_params(p);
  if (!e.empty()) return fail(nullptr, COG_E_INVALID, e);
  if (!bytes) return fail(nullptr, COG_E_INVALID, "bytes is NULL");
  const size_t P = (size_t)p->width * p->height, C = (size_t)p->channels, K = (size_t)p->K;
  *bytes = 64 + pad64(P * K * (C + 2) * 4) + pad64(P * (C + 1) * 4) + pad64(P * C * 16) +
           pad64(P * 3 * 2) + pad64(P) + pad64(P * C * 4) + pad64(P * 2) + pad64(P * 8) + pad64(P);
  return COG_OK;
}

cog_status cog_kde_weights(float h, uint16_t *out) {
  if (!out) return fail(nullptr, COG_E_INVALID, "out is NULL");
  if (!(h > 0.0f)) return fail(nullptr, COG_E_INVALID, "bandwidth must be positive");
  kde_table((double)h, out);
  return COG_OK;
}

cog_status cog_create(const cog_params *p, void *hip_stream, void *device_state,
                      size_t state_bytes, cog_ctx **out) {
  if (!out) return fail(nullptr, COG_E_INVALID, "out is NULL");
  *out = nullptr;
  const std::string e = check_params(p);
  if (!e.empty()) return fail(nullptr, COG_E_INVALID, e);
  if ((p->stage_mask & COG_STAGE_SAMPLE) && p->tile_px != 0 && p->tile_px != 64)
    return fail(nullptr, COG_E_UNSUPPORTED, "sampling runs with 64-pixel tiles only");
  const Plan pl = make_plan(p);
  if (device_state && (reinterpret_cast<uintptr_t>(device_state) & 255))
    return fail(nullptr, COG_E_INVALID, "device_state must be 256-byte aligned");
  if (device_state && state_bytes < pl.total)
    return fail(nullptr, COG_E_OOM, "device_state smaller than cog_state_bytes()");

  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    return fail(nullptr, COG_E_DEVICE, std::string("no HIP device: ") + hipGetErrorString(he));
  }
  cog_ctx *h = new (std::nothrow) cog_ctx();
  if (!h) return fail(nullptr, COG_E_OOM, "host allocation failed");
  h->p = *p;
  h->plan = pl;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->device = dev;
  if (device_state) {
    h->dstate = static_cast<char *>(device_state);
  } else {
    he = hipMalloc((void **)&h->dstate, pl.total);
    if (he != hipSuccess) {
      delete h;
      return fail(nullptr, COG_E_OOM, "state allocation failed");
    }
    h->own_state = true;
  }
  h->buf.gmm = reinterpret_cast<float *>(h->dstate + pl.off_gmm);
  h->buf.rga = reinterpret_cast<float *>(h->dstate + pl.off_rga);
  h->buf.prior = reinterpret_cast<uint8_t *>(h->dstate + pl.off_prior);
  h->buf.cnt = reinterpret_cast<uint16_t *>(h->dstate + pl.off_cnt);
  h->buf.prev = h->dstate + pl.off_prev;
  h->buf.labels = reinterpret_cast<unsigned long long *>(h->dstate + pl.off_labels);
  h->buf.kdew = reinterpret_cast<const uint16_t *>(h->dstate + pl.off_kdew);
  h->buf.sat = reinterpret_cast<uint16_t *>(h->dstate + pl.off_sat);
  h->buf.gkey = reinterpret_cast<uint2 *>(h->dstate + pl.off_gkey);
  h->buf.P = pl.P;

  // prior kernel weights, uploaded level-major [256][16]
  std::vector<uint16_t> W(16 * 256), Wt(16 * 256);
  kde_table((double)p->kde_h, W.data());
  for (int b = 0; b < 16; ++b)
    for (int v = 0; v < 256; ++v) Wt[v * 16 + b] = W[b * 256 + v];
  he = hipMemcpyAsync(h->dstate + pl.off_kdew, Wt.data(), Wt.size() * 2, hipMemcpyHostToDevice,
                      h->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(h->stream);
  if (he != hipSuccess) {
    cog_status s = hip_fail(nullptr, he, "weight upload");
    if (h->own_state) (void)hipFree(h->dstate);
    delete h;
    return s;
  }
  h->kp = make_kparams(p, 2);
  // the device address of this GPU's no-allocation scratch, looked up while
  // the GPU is current (only cog_group_background_noalloc needs it)
  he = cog::scratch_for_device(dev, &h->scratch);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    h->scratch = nullptr;
    h->scratch_err = hipGetErrorString(he);
  }
  *out = h;
  return COG_OK;
}

cog_status cog_train_prior(cog_ctx *h, const void *frames, int32_t n, int32_t frames_on_device) {
  if (!h) return fail(nullptr, COG_E_INVALID, "context is NULL");
  if (!frames) return fail(h, COG_E_INVALID, "frames is NULL");
  if (n < 2 || n > 65536) return fail(h, COG_E_INVALID, "training needs 2 <= n <= 65536 frames");
  if (h->n_train != 0) return fail(h, COG_E_STATE, "already trained");
  const Plan &pl = h->plan;
  const size_t fbytes = (size_t)pl.P * pl.C * pl.sin;
  const void *dfr = frames;
  if (!frames_on_device) {
    cog_status s = ensure_stage(h, fbytes * n, 0);
    if (s != COG_OK) return s;
    hipError_t e = hipMemcpyAsync(h->stage_in, frames, fbytes * n, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "frame upload");
    dfr = h->stage_in;
  }
  cog_status s = cog_rt::train_range(h, dfr, n, 0, pl.P, h->stream);
  if (s != COG_OK) return s;
  if (!frames_on_device) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "training");
  }
  cog_rt::train_finish(h, n);
  return COG_OK;
}

extern "C++" {
namespace cog_rt {

cog_status train_range(cog_ctx *h, const void *dframes, int n, int64_t p0, int64_t p1,
                       hipStream_t st) {
  const Plan &pl = h->plan;
  const cog::KParams kp = make_kparams(&h->p, n);
  const bool cascade = h->p.path == COG_PATH_CASCADE;
  hipError_t e = cog::launch_train(pl.C, pl.K, h->p.dtype == COG_F32, cascade, cascade, h->buf,
                                   dframes, (int64_t)pl.P * pl.C, n, kp, p0, p1, st);
  if (e != hipSuccess) return hip_fail(h, e, "training launch");
  return COG_OK;
}

void train_finish(cog_ctx *h, int n) {
  h->kp = make_kparams(&h->p, n);
  h->n_train = n;
  h->frame = n;
}

}  // namespace cog_rt
}  // extern "C++"

cog_status cog_step_frames(cog_ctx *h, const void *frames, int32_t n, int32_t frames_on_device,
                           uint8_t *masks_out, int32_t masks_on_device, cog_step_info *infos) {
  if (!h) return fail(nullptr, COG_E_INVALID, "context is NULL");
  if (!frames) return fail(h, COG_E_INVALID, "frames is NULL");
  if (n < 1) return fail(h, COG_E_INVALID, "n must be >= 1");
  if (h->n_train == 0) return fail(h, COG_E_STATE, "cog_train_prior has not run");
  const Plan &pl = h->plan;
  const size_t fbytes = (size_t)pl.P * pl.C * pl.sin;
  const size_t mbytes = (size_t)pl.P;
  const bool host_in = !frames_on_device;
  const bool host_mask = masks_out && !masks_on_device;
  cog_status s = ensure_stage(h, host_in ? fbytes * n : 0, host_mask ? mbytes * n : 0);
  if (s != COG_OK) return s;
  const void *dfr = frames;
  if (host_in) {
    hipError_t e = hipMemcpyAsync(h->stage_in, frames, fbytes * n, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "frame upload");
    dfr = h->stage_in;
  }
  uint8_t *dm = host_mask ? h->stage_mask : masks_out;
  s = run_frames(h, dfr, n, dm, infos != nullptr, infos);
  if (s != COG_OK) return s;
  if (host_mask) {
    hipError_t e = hipMemcpyAsync(masks_out, h->stage_mask, mbytes * n, hipMemcpyDeviceToHost,
                                  h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "mask download");
  } else if (host_in) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "step");
  }
  h->frame += n;
  return COG_OK;
}

cog_status cog_step(cog_ctx *h, const void *frame, int32_t frame_on_device, uint8_t *mask_out,
                    int32_t mask_on_device, cog_step_info *info) {
  return cog_step_frames(h, frame, 1, frame_on_device, mask_out, mask_on_device, info);
}

cog_status cog_reset(cog_ctx *h) {
  if (!h) return fail(nullptr, COG_E_INVALID, "context is NULL");
  h->n_train = 0;
  h->frame = 0;
  h->kp = make_kparams(&h->p, 2);
  return COG_OK;
}

void cog_destroy(cog_ctx *h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  if (h->own_state && h->dstate) (void)hipFree(h->dstate);
  if (h->stage_in) (void)hipFree(h->stage_in);
  if (h->stage_mask) (void)hipFree(h->stage_mask);
  if (h->rows_ws) (void)hipFree(h->rows_ws);
  delete h;
}

cog_status cog_export_state(cog_ctx *h, void *host_dst, size_t bytes) {
  if (!h) return fail(nullptr, COG_E_INVALID, "context is NULL");
  if (!host_dst) return fail(h, COG_E_INVALID, "host_dst is NULL");
  size_t need = 0;
  cog_canonical_bytes(&h->p, &need);
  if (bytes < need) return fail(h, COG_E_INVALID, "buffer smaller than cog_canonical_bytes()");
  const Plan &pl = h->plan;
  std::vector<char> raw(pl.off_kdew);
  hipError_t e = hipMemcpyAsync(raw.data(), h->dstate, raw.size(), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "state download");

  const size_t P = (size_t)pl.P, C = (size_t)pl.C, K = (size_t)pl.K;
  char *o = static_cast<char *>(host_dst);
  std::memset(o, 0, need);
  const uint32_t h32[2] = {kMagic, 3u};
  const int32_t hi[6] = {h->p.width, h->p.height, h->p.channels, h->p.K, h->p.dtype, h->n_train};
  std::memcpy(o, h32, 8);
  std::memcpy(o + 8, hi, 24);
  std::memcpy(o + 32, &h->frame, 8);
  size_t off = 64;
  float *g = reinterpret_cast<float *>(o + off);
  const float *rg = reinterpret_cast<const float *>(raw.data() + pl.off_gmm);
  const bool aos = h->p.path == COG_PATH_CASCADE;
  for (size_t p = 0; p < P; ++p) {
    for (size_t k = 0; k < K; ++k) {
      for (size_t f = 0; f < C + 2; ++f) {
        // canonical field f: 0 = w, 1..C = mu, C+1 = var
        size_t fld = f == 0 ? k : (f == C + 1 ? K + k : 2 * K + k * C + (f - 1));
        size_t idx = aos ? p * pl.R + fld : ((p >> 6) * pl.R + fld) * 64 + (p & 63);
        g[(p * K + k) * (C + 2) + f] = rg[idx];
      }
    }
  }
  off += pad64(P * K * (C + 2) * 4);
  if (aos) {
    // the stored variance carries the pixel's shared flag in its sign bit
    const uint32_t *rr = reinterpret_cast<const uint32_t *>(raw.data() + pl.off_rga);
    uint32_t *r = reinterpret_cast<uint32_t *>(o + off);
    for (size_t p = 0; p < P; ++p)
      for (size_t c = 0; c <= C; ++c)
        r[p * (C + 1) + c] = rr[p * pl.RG + c] & (c == C ? 0x7fffffffu : 0xffffffffu);
  }
  off += pad64(P * (C + 1) * 4);
  if (aos) {
    const uint8_t *pr = reinterpret_cast<const uint8_t *>(raw.data() + pl.off_prior);
    uint8_t *t = reinterpret_cast<uint8_t *>(o + off);
    for (size_t p = 0; p < P; ++p) std::memcpy(t + p * C * 16, pr + p * pl.PB, C * 16);
    off += pad64(P * C * 16);
    const uint16_t *cs = reinterpret_cast<const uint16_t *>(raw.data() + pl.off_cnt);
    uint16_t *cn = reinterpret_cast<uint16_t *>(o + off);
    for (size_t p = 0; p < P; ++p) std::memcpy(cn + p * 3, cs + p * 4, 6);
    off += pad64(P * 3 * 2);
  } else {
    off += pad64(P * C * 16) + pad64(P * 3 * 2);
  }
  const uint64_t *lw = reinterpret_cast<const uint64_t *>(raw.data() + pl.off_labels);
  uint8_t *lb = reinterpret_cast<uint8_t *>(o + off);
  for (size_t p = 0; p < P; ++p) lb[p] = (uint8_t)((lw[p >> 6] >> (p & 63)) & 1u);
  off += pad64(P);
  float *pv = reinterpret_cast<float *>(o + off);
  for (size_t i = 0; i < P * C; ++i) {
    if (pl.sin == 1) pv[i] = (float)reinterpret_cast<const uint8_t *>(raw.data() + pl.off_prev)[i];
    else pv[i] = reinterpret_cast<const float *>(raw.data() + pl.off_prev)[i];
  }
  off += pad64(P * C * 4);
  if (aos) std::memcpy(o + off, raw.data() + pl.off_sat, P * 2);
  off += pad64(P * 2);
  if (aos) std::memcpy(o + off, raw.data() + pl.off_gkey, P * 8);
  off += pad64(P * 8);
  if (aos) {
    const uint32_t *rr = reinterpret_cast<const uint32_t *>(raw.data() + pl.off_rga);
    uint8_t *sh = reinterpret_cast<uint8_t *>(o + off);
    for (size_t p = 0; p < P; ++p) sh[p] = (uint8_t)(rr[p * pl.RG + C] >> 31);
  }
  return COG_OK;
}

cog_status cog_import_state(cog_ctx *h, const void *host_src, size_t bytes) {
  if (!h) return fail(nullptr, COG_E_INVALID, "context is NULL");
  if (!host_src) return fail(h, COG_E_INVALID, "host_src is NULL");
  if (bytes < 64) return fail(h, COG_E_INVALID, "buffer smaller than a canonical header");
  const char *in = static_cast<const char *>(host_src);
  uint32_t ver = 0;
  std::memcpy(&ver, in + 4, 4);
  size_t need = 0;
  cog_canonical_bytes(&h->p, &need);
  // version 1 has no saturation, grouping-key and shared sections, version 2
  // no shared section
  if (ver <= 2u) need -= pad64((size_t)h->plan.P);
  if (ver == 1u) need -= pad64((size_t)h->plan.P * 2) + pad64((size_t)h->plan.P * 8);
  if (bytes < need) return fail(h, COG_E_INVALID, "buffer smaller than the canonical state");
  uint32_t h32[2];
  int32_t hi[6];
  int64_t frame;
  std::memcpy(h32, in, 8);
  std::memcpy(hi, in + 8, 24);
  std::memcpy(&frame, in + 32, 8);
  if (h32[0] != kMagic || h32[1] < 1u || h32[1] > 3u)
    return fail(h, COG_E_INVALID, "not a canonical state");
  if (hi[0] != h->p.width || hi[1] != h->p.height || hi[2] != h->p.channels || hi[3] != h->p.K ||
      hi[4] != h->p.dtype)
    return fail(h, COG_E_INVALID, "state shape does not match the context");
  if (hi[5] < 2 || hi[5] > 65536) return fail(h, COG_E_INVALID, "state has no training");
  const Plan &pl = h->plan;
  std::vector<char> raw(pl.off_kdew, 0);
  const size_t P = (size_t)pl.P, C = (size_t)pl.C, K = (size_t)pl.K;
  size_t off = 64;
  const float *g = reinterpret_cast<const float *>(in + off);
  float *rg = reinterpret_cast<float *>(raw.data() + pl.off_gmm);
  const bool aos = h->p.path == COG_PATH_CASCADE;
  for (size_t p = 0; p < P; ++p)
    for (size_t k = 0; k < K; ++k)
      for (size_t f = 0; f < C + 2; ++f) {
        size_t fld = f == 0 ? k : (f == C + 1 ? K + k : 2 * K + k * C + (f - 1));
        size_t idx = aos ? p * pl.R + fld : ((p >> 6) * pl.R + fld) * 64 + (p & 63);
        rg[idx] = g[(p * K + k) * (C + 2) + f];
      }
  off += pad64(P * K * (C + 2) * 4);
  if (aos) {
    const uint32_t *r = reinterpret_cast<const uint32_t *>(in + off);
    uint32_t *rr = reinterpret_cast<uint32_t *>(raw.data() + pl.off_rga);
    for (size_t p = 0; p < P; ++p)
      for (size_t c = 0; c <= C; ++c)
        rr[p * pl.RG + c] = r[p * (C + 1) + c] & (c == C ? 0x7fffffffu : 0xffffffffu);
  }
  off += pad64(P * (C + 1) * 4);
  if (aos) {
    uint8_t *pr = reinterpret_cast<uint8_t *>(raw.data() + pl.off_prior);
    const uint8_t *t = reinterpret_cast<const uint8_t *>(in + off);
    for (size_t p = 0; p < P; ++p) std::memcpy(pr + p * pl.PB, t + p * C * 16, C * 16);
    off += pad64(P * C * 16);
    const uint16_t *cn = reinterpret_cast<const uint16_t *>(in + off);
    uint16_t *cs = reinterpret_cast<uint16_t *>(raw.data() + pl.off_cnt);
    const float nm1 = (float)(hi[5] - 1);
    for (size_t p = 0; p < P; ++p) {
      std::memcpy(cs + p * 4, cn + p * 3, 6);
      // confidence weights as the training kernel stores them
      float abg[3];
      for (int i = 0; i < 3; ++i) abg[i] = (float)cn[p * 3 + i] / nm1;
      std::memcpy(pr + p * pl.PB + C * 16, abg, 12);
    }
    off += pad64(P * 3 * 2);
  } else {
    off += pad64(P * C * 16) + pad64(P * 3 * 2);
  }
  const uint8_t *lb = reinterpret_cast<const uint8_t *>(in + off);
  uint64_t *lw = reinterpret_cast<uint64_t *>(raw.data() + pl.off_labels);
  for (size_t p = 0; p < P; ++p)
    if (lb[p]) lw[p >> 6] |= (uint64_t)1 << (p & 63);
  off += pad64(P);
  const float *pv = reinterpret_cast<const float *>(in + off);
  for (size_t i = 0; i < P * C; ++i) {
    if (pl.sin == 1) {
      float v = pv[i];
      if (!(v >= 0.0f && v <= 255.0f) || v != std::floor(v))
        return fail(h, COG_E_INVALID, "previous frame is not on the u8 level grid");
      reinterpret_cast<uint8_t *>(raw.data() + pl.off_prev)[i] = (uint8_t)v;
    } else {
      reinterpret_cast<float *>(raw.data() + pl.off_prev)[i] = pv[i];
    }
  }
  off += pad64(P * C * 4);
  if (aos && ver >= 2u) std::memcpy(raw.data() + pl.off_sat, in + off, P * 2);
  off += pad64(P * 2);
  if (aos && ver >= 2u) std::memcpy(raw.data() + pl.off_gkey, in + off, P * 8);
  off += pad64(P * 8);
  if (aos && ver >= 3u) {
    const uint8_t *sh = reinterpret_cast<const uint8_t *>(in + off);
    uint32_t *rr = reinterpret_cast<uint32_t *>(raw.data() + pl.off_rga);
    for (size_t p = 0; p < P; ++p)
      if (sh[p]) rr[p * pl.RG + C] |= 0x80000000u;
  }
  hipError_t e = hipMemcpyAsync(h->dstate, raw.data(), raw.size(), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "state upload");
  h->n_train = hi[5];
  h->frame = frame;
  h->kp = make_kparams(&h->p, h->n_train);
  return COG_OK;
}

cog_status cog_group_share(cog_ctx *h, const uint8_t *map, int32_t map_on_device,
                           float *gvar_out) {
  cog_status s = group_check(h);
  if (s != COG_OK) return s;
  const Plan &pl = h->plan;
  const int64_t P = pl.P;
  const int nb = cog::group_blocks(P);
  constexpr int W = 2 * cog::kGroups + 1;
  hipStream_t st = h->stream;
  uint8_t *dmap = nullptr;
  uint64_t *part = nullptr;
  const bool copy_map = map && !map_on_device;
  if ((copy_map && hipMalloc((void **)&dmap, (size_t)P) != hipSuccess) ||
      hipMalloc((void **)&part, ((size_t)nb * W + W) * 8) != hipSuccess) {
    (void)hipGetLastError();
    if (dmap) (void)hipFree(dmap);
    return fail(h, COG_E_OOM, "sharing scratch allocation failed");
  }
  cog_status rc = COG_OK;
  auto check = [&](hipError_t e, const char *what) {
    if (e != hipSuccess && rc == COG_OK) rc = hip_fail(h, e, what);
    return rc == COG_OK;
  };
  const uint8_t *m = copy_map ? dmap : map;
  cog::ShareVars v{};
  if (map) {
    uint64_t row[W] = {0};
    if (copy_map) check(hipMemcpyAsync(dmap, map, (size_t)P, hipMemcpyHostToDevice, st), "copy");
    if (rc == COG_OK &&
        check(cog::launch_share_sum(h->buf.rga, pl.RG, pl.C, P, m, part, st), "sharing launch") &&
        check(cog::launch_part_reduce(part, nb, W, 0u, 0u, part + (size_t)nb * W, st),
              "sharing launch") &&
        check(hipMemcpyAsync(row, part + (size_t)nb * W, sizeof(row), hipMemcpyDeviceToHost, st),
              "copy"))
      check(hipStreamSynchronize(st), "sharing");
    if (rc == COG_OK && row[W - 1] != 0)
      rc = fail(h, COG_E_INVALID, "group map holds a value other than 0..2 and 255, or a variance "
                                  "beyond 2^37");
    // the exact member mean on the 2^-16 grid, one binary64 division, then
    // binary32, held at var_min or above
    for (int g = 0; rc == COG_OK && g < cog::kGroups; ++g) {
      if (!row[2 * g]) continue;
      const float mean = (float)((double)row[2 * g + 1] / 65536.0 / (double)row[2 * g]);
      v.var[g] = mean < h->p.var_min ? h->p.var_min : mean;
    }
  }
  if (rc == COG_OK) {
    check(cog::launch_share_set(h->buf.rga, pl.RG, pl.C, P, m, v, st), "sharing launch");
    check(hipStreamSynchronize(st), "sharing");
  }
  (void)hipStreamSynchronize(st);
  if (dmap) (void)hipFree(dmap);
  (void)hipFree(part);
  if (rc == COG_OK && gvar_out)
    for (int g = 0; g < cog::kGroups; ++g) gvar_out[g] = v.var[g];
  return rc;
}

cog_status cog_group_background(cog_ctx *h, uint8_t *map_out, int32_t map_on_device,
                                cog_group_info *info) {
  cog_status s = group_check(h);
  if (s != COG_OK) return s;
  const int64_t P = h->plan.P;
  const size_t part_words = (size_t)cog::group_blocks(P) * cog::kGroupStat;
  uint8_t *asg = nullptr;
  uint64_t *part = nullptr;
  if (hipMalloc((void **)&asg, (size_t)P * 2) != hipSuccess ||
      hipMalloc((void **)&part, (part_words + cog::kGroupStat) * 8) != hipSuccess) {
    (void)hipGetLastError();
    if (asg) (void)hipFree(asg);
    return fail(h, COG_E_OOM, "grouping scratch allocation failed");
  }
  s = group_run(h, map_out, map_on_device, info, asg, asg + P, part, part + part_words);
  (void)hipStreamSynchronize(h->stream);
  (void)hipFree(asg);
  (void)hipFree(part);
  return s;
}

cog_status cog_group_background_noalloc(cog_ctx *h, uint8_t *map_out, int32_t map_on_device,
                                        cog_group_info *info) {
  cog_status s = group_check(h);
  if (s != COG_OK) return s;
  if (h->plan.P > cog::kNoAllocMaxPixels)
    return fail(h, COG_E_INVALID, "frame larger than the no-allocation scratch (at most " +
                                      std::to_string(cog::kNoAllocMaxPixels) + " pixels)");
  char *sc = h->scratch;
  if (!sc) return fail(h, COG_E_DEVICE, "no-allocation scratch unavailable: " + h->scratch_err);
  return group_run(h, map_out, map_on_device, info, reinterpret_cast<uint8_t *>(sc + cog::kScratchAsg),
                   reinterpret_cast<uint8_t *>(sc + cog::kScratchMap),
                   reinterpret_cast<uint64_t *>(sc + cog::kScratchPart),
                   reinterpret_cast<uint64_t *>(sc + cog::kScratchRed));
}

const char *cog_last_error(const cog_ctx *h) {
  if (h) return h->err.c_str();
  return g_err.c_str();
}

}  // extern "C"
