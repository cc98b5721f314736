// Host runtime of the batched tick (include/cog.h, "Batched tick").
//
// A tick groups its items by class (channels, K, input type); each class
// gets one persistent launch of k_tick over the concatenated 64-pixel tiles
// of its streams -- or, when the class's schedule compacts, its items that
// advance by one frame get a launch of their own, k_tick_c over 256-pixel
// tiles whose survivors are compacted per wave.  The per-item descriptors (frames, state pointers,
// parameters, first tile) are written to pinned host memory and copied to a
// fixed device region per class position, so a captured hipGraph of the
// tick's launches stays valid from tick to tick and is replayed whenever the
// classes, their schedules and grid sizes repeat.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <set>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "cog.h"
#include "cog_ctx.h"
#include "cog_device.h"

namespace {

constexpr int kMaxClasses = 8;     // classes in one tick
constexpr int kMaxLaunches = 2 * kMaxClasses;  // a compacting and a plain launch per class
constexpr int kMaxGraphs = 64;     // cached graph executables
constexpr int kMaxSeen = 256;      // launch sets remembered for capture on reuse
constexpr int kMaxItemsLimit = 4096;

// A class of streams shares one kernel instantiation: channels, K, input
// type, and whether sampling is on.  Schedules are set per (C, K, f32).
struct ClassKey {
  int C, K, f32, samp;
  bool operator<(const ClassKey &o) const {
    return std::tie(C, K, f32, samp) < std::tie(o.C, o.K, o.f32, o.samp);
  }
  ClassKey sched_key() const { return ClassKey{C, K, f32, 0}; }
};

ClassKey class_of(const cog_ctx *h) {
  return ClassKey{h->plan.C, h->plan.K, h->p.dtype == COG_F32 ? 1 : 0,
                  (h->p.stage_mask & COG_STAGE_SAMPLE) ? 1 : 0};
}

// One class's launch in a tick.
struct Launch {
  ClassKey key;
  bool compact = false;  // k_tick_c over kFrameTile-pixel tiles (one frame per item)
  bool lp = false;
  int grid = 0;
  int dynamic = 0;
  int group = 1;
  bool graph = true;
  std::vector<int> items;  // indices into the caller's item array
  int64_t tiles = 0;
};

struct GraphEntry {
  std::vector<int64_t> key;
  hipGraphExec_t exec = nullptr;
  uint64_t used = 0;
};

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Workgroup counts rounded up to one of eight steps per octave (at most 1/8
// of the workgroups find no unit and exit at once), so that ticks of varying
// size share a few launch shapes and hence a few captured graphs.
int64_t grid_bucket(int64_t n) {
  if (n <= 16) return n;
  int top = 63;
  while (!((n >> top) & 1)) --top;
  const int64_t q = (int64_t)1 << (top - 3);
  return (n + q - 1) / q * q;
}

}  // namespace

struct cog_batch {
  hipStream_t stream = nullptr;
  int device = 0;
  int ncu = 0;
  int max_items = 0;
  size_t region_bytes = 0;   // head + max_items items
  char *ddesc = nullptr;     // kMaxLaunches regions, then the statistics job table
  size_t desc_bytes = 0;
  char *hdesc[2] = {nullptr, nullptr};
  hipEvent_t hev[2] = {nullptr, nullptr};
  bool hev_used[2] = {false, false};
  int hcur = 0;
  uint32_t *dstat = nullptr;
  size_t dstat_cap = 0;      // u32 words
  std::vector<uint32_t> hstat;
  std::map<ClassKey, cog_schedule> sched;
  std::map<std::tuple<int, int, int, int, int>, int> occ;
  std::vector<GraphEntry> graphs;
  // launch sets seen once and not captured yet (most recent last)
  std::vector<std::vector<int64_t>> seen;
  uint64_t use_clock = 0;
};

namespace {

using cog_rt::fail;
using cog_rt::hip_fail;

cog_status bfail(cog_status s, const std::string &msg) { return fail(nullptr, s, msg); }
cog_status bhip(hipError_t e, const char *what) {
  return bfail(COG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Measured on MI355X over a 64-stream mixed workload: handing units of 4
// tiles to the hardware dispatcher matches or beats every persistent grid,
// and the atomic queue (one counter shared by every wave of the chip) is
// several times slower than either.
cog_schedule default_schedule() {
  cog_schedule s;
  s.blocks_per_cu = -1;
  s.dynamic = 0;
  s.group = 4;
  s.use_graph = 1;
  s.compact = 1;
  return s;
}

// Tiles of one item in a launch.
int64_t item_tiles(const cog_ctx *h, bool compact) {
  return compact ? (h->plan.P + cog::kFrameTile - 1) / cog::kFrameTile : h->plan.ntiles;
}

std::string check_schedule(const cog_schedule *s) {
  if (!s) return "schedule is NULL";
  if (s->blocks_per_cu < -1 || s->blocks_per_cu > 64) return "blocks_per_cu must be in [-1, 64]";
  if (s->dynamic != 0 && s->dynamic != 1) return "dynamic must be 0 or 1";
  if (s->group < 1 || s->group > 1024) return "group must be in [1, 1024]";
  if (s->use_graph != 0 && s->use_graph != 1) return "use_graph must be 0 or 1";
  if (s->compact != 0 && s->compact != 1) return "compact must be 0 or 1";
  return std::string();
}

int occupancy(cog_batch *b, const ClassKey &k, bool lp, bool compact) {
  const auto key = std::make_tuple(k.C, k.K, k.f32, k.samp, compact ? 2 : (lp ? 1 : 0));
  auto it = b->occ.find(key);
  if (it != b->occ.end()) return it->second;
  int n = compact ? cog::tick_c_blocks_per_cu(k.C, k.K, k.f32 != 0)
                  : cog::tick_blocks_per_cu(k.C, k.K, k.f32 != 0, lp, k.samp != 0);
  if (n < 1) n = 1;
  b->occ[key] = n;
  return n;
}

// Validation shared by tick and autotune; fills the active items' launches.
cog_status plan_tick(cog_batch *b, const cog_tick_item *items, int32_t n, bool want_infos,
                     std::vector<Launch> &launches, bool &any_infos) {
  launches.clear();
  any_infos = false;
  if (!b) return bfail(COG_E_INVALID, "batch is NULL");
  if (n < 0 || n > b->max_items) return bfail(COG_E_INVALID, "item count out of range");
  if (n > 0 && !items) return bfail(COG_E_INVALID, "items is NULL");
  std::vector<const cog_ctx *> seen;
  seen.reserve(n);
  // an item's launch: its class, compacting when the class's schedule says
  // so and the item advances by one frame without sampling
  auto compact_of = [&](const cog_tick_item &it) {
    const ClassKey key = class_of(it.ctx);
    if (key.samp || it.nframes != 1) return false;
    auto sit = b->sched.find(key.sched_key());
    return (sit == b->sched.end() ? default_schedule() : sit->second).compact != 0;
  };
  std::map<std::pair<ClassKey, bool>, int> pos;
  std::map<ClassKey, int> classes;
  for (int i = 0; i < n; ++i) {
    const cog_tick_item &it = items[i];
    cog_ctx *h = it.ctx;
    if (!h) return bfail(COG_E_INVALID, "item has no context");
    if (it.nframes < 0) return bfail(COG_E_INVALID, "nframes must be >= 0");
    if (it.reserved != 0) return bfail(COG_E_INVALID, "reserved must be 0");
    if (h->stream != b->stream) return bfail(COG_E_INVALID, "context is not on the batch's stream");
    if (h->p.path != COG_PATH_CASCADE) return bfail(COG_E_UNSUPPORTED, "batched ticks run the cascade path only");
    if (h->plan.tile != 64) return bfail(COG_E_UNSUPPORTED, "batched ticks need 64-pixel tiles");
    if (h->n_train == 0) return bfail(COG_E_STATE, "context is not trained");
    seen.push_back(h);
    if (it.nframes == 0) continue;
    if (!it.frames) return bfail(COG_E_INVALID, "frames is NULL");
    if (want_infos && it.infos) {
      if (it.nframes > h->plan.stat_chunk)
        return bfail(COG_E_INVALID, "too many frames for one item with infos (the stream's statistics "
                                    "workspace holds " + std::to_string(h->plan.stat_chunk) + ")");
      any_infos = true;
    }
    const ClassKey key = class_of(h);
    if (classes.find(key) == classes.end()) {
      if ((int)classes.size() == kMaxClasses) return bfail(COG_E_INVALID, "more than 8 classes in one tick");
      classes[key] = 0;
    }
    pos[std::make_pair(key, compact_of(it))] = -1;
  }
  std::sort(seen.begin(), seen.end());
  if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
    return bfail(COG_E_INVALID, "a context appears twice in one tick");
  // classes in key order, items in caller order within a class
  int j = 0;
  for (auto &kv : pos) kv.second = j++;
  launches.resize(pos.size());
  for (auto &kv : pos) {
    launches[kv.second].key = kv.first.first;
    launches[kv.second].compact = kv.first.second;
  }
  for (int i = 0; i < n; ++i) {
    if (items[i].nframes == 0) continue;
    const bool c = compact_of(items[i]);
    Launch &L = launches[pos[std::make_pair(class_of(items[i].ctx), c)]];
    L.items.push_back(i);
    L.tiles += item_tiles(items[i].ctx, c);
  }
  for (Launch &L : launches) {
    if (L.tiles > 0x7fffffff) return bfail(COG_E_INVALID, "a tick's class exceeds 2^31 tiles");
    int minf = 1 << 30;
    for (int i : L.items) minf = std::min(minf, items[i].nframes);
    L.lp = minf >= 8;
    auto sit = b->sched.find(L.key.sched_key());
    const cog_schedule s = sit == b->sched.end() ? default_schedule() : sit->second;
    L.group = s.group;
    L.graph = s.use_graph != 0;
    const int64_t units = (L.tiles + s.group - 1) / s.group;
    if (s.blocks_per_cu < 0) {
      const int64_t g = grid_bucket(units);
      if (g > 0x7fffffff) return bfail(COG_E_INVALID, "tick too large for one workgroup per unit");
      L.grid = (int)g;
      L.dynamic = 0;
    } else {
      const int bpc = s.blocks_per_cu == 0 ? occupancy(b, L.key, L.lp, L.compact) : s.blocks_per_cu;
      const int64_t cap = (int64_t)bpc * b->ncu;
      L.grid = (int)(units >= cap ? cap : std::min(cap, grid_bucket(units)));
      L.dynamic = s.dynamic;
    }
    if (L.grid < 1) L.grid = 1;
  }
  return COG_OK;
}

cog::TickHead *region_head(cog_batch *b, char *base, int j) {
  return reinterpret_cast<cog::TickHead *>(base + (size_t)j * b->region_bytes);
}
cog::TickItem *region_items(cog_batch *b, char *base, int j) {
  return reinterpret_cast<cog::TickItem *>(base + (size_t)j * b->region_bytes + sizeof(cog::TickHead));
}

cog_status launch_all(cog_batch *b, const std::vector<Launch> &launches) {
  for (size_t j = 0; j < launches.size(); ++j) {
    const Launch &L = launches[j];
    hipError_t e = L.compact
        ? cog::launch_tick_c(L.key.C, L.key.K, L.key.f32 != 0, region_head(b, b->ddesc, (int)j),
                             region_items(b, b->ddesc, (int)j), L.grid, L.dynamic, b->stream)
        : cog::launch_tick(L.key.C, L.key.K, L.key.f32 != 0, L.lp, L.key.samp != 0,
                           region_head(b, b->ddesc, (int)j), region_items(b, b->ddesc, (int)j),
                           L.grid, L.dynamic, b->stream);
    if (e != hipSuccess) return bhip(e, "tick launch");
  }
  return COG_OK;
}

// Replays (capturing on first use) the graph of this launch list.
cog_status run_graph(cog_batch *b, const std::vector<Launch> &launches) {
  std::vector<int64_t> key;
  for (const Launch &L : launches) {
    key.push_back(L.key.C);
    key.push_back(L.key.K);
    key.push_back(L.key.f32);
    key.push_back(L.key.samp);
    key.push_back(L.compact);
    key.push_back(L.lp);
    key.push_back(L.grid);
    key.push_back(L.dynamic);
  }
  GraphEntry *ge = nullptr;
  for (GraphEntry &g : b->graphs)
    if (g.key == key) ge = &g;
  if (!ge) {
    // a launch set is captured the second time it occurs: one-off sets (a
    // serving tick of unusual size) launch directly instead of paying for an
    // instantiation they would never reuse
    auto it = std::find(b->seen.begin(), b->seen.end(), key);
    if (it == b->seen.end()) {
      if ((int)b->seen.size() == kMaxSeen) b->seen.erase(b->seen.begin());
      b->seen.push_back(key);
      return launch_all(b, launches);
    }
    b->seen.erase(it);
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bhip(e, "graph capture");
    cog_status s = launch_all(b, launches);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->stream, &g);
    if (s != COG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return bhip(e, "graph capture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return bhip(e, "graph instantiation");
    if ((int)b->graphs.size() == kMaxGraphs) {
      auto lru = std::min_element(b->graphs.begin(), b->graphs.end(),
                                  [](const GraphEntry &x, const GraphEntry &y) { return x.used < y.used; });
      (void)hipGraphExecDestroy(lru->exec);
      b->graphs.erase(lru);
    }
    b->graphs.push_back(GraphEntry{key, ex, 0});
    ge = &b->graphs.back();
  }
  ge->used = ++b->use_clock;
  hipError_t e = hipGraphLaunch(ge->exec, b->stream);
  if (e != hipSuccess) return bhip(e, "graph launch");
  return COG_OK;
}

// Writes the descriptors, uploads them and runs the launches; with stats,
// reduces the counters of the items that asked and fills their infos.
cog_status execute(cog_batch *b, const cog_tick_item *items, const std::vector<Launch> &launches,
                   bool stats) {
  const int cur = b->hcur;
  if (b->hev_used[cur]) {
    hipError_t e = hipEventSynchronize(b->hev[cur]);
    if (e != hipSuccess) return bhip(e, "descriptor staging");
  }
  char *hb = b->hdesc[cur];
  std::vector<cog::StatJob> jobs;
  std::vector<size_t> job_item, job_off;
  std::vector<int> job_blk;
  size_t stat_words = 0;
  int max_blk = 0, max_fr = 0;
  for (size_t j = 0; j < launches.size(); ++j) {
    const Launch &L = launches[j];
    cog::TickHead *hh = region_head(b, hb, (int)j);
    std::memset(hh, 0, sizeof(*hh));
    hh->total_tiles = L.tiles;
    hh->n_items = (int32_t)L.items.size();
    hh->group = L.group;
    hh->queue = 0u;
    cog::TickItem *ti = region_items(b, hb, (int)j);
    int64_t tb = 0;
    for (size_t q = 0; q < L.items.size(); ++q) {
      const cog_tick_item &it = items[L.items[q]];
      const cog_ctx *h = it.ctx;
      cog::TickItem &d = ti[q];
      std::memset(&d, 0, sizeof(d));
      d.fr.x = it.frames;
      d.fr.stride = h->plan.P * h->plan.C;
      d.fr.mask = it.masks;
      d.fr.mstride = h->plan.P;
      const bool want = stats && it.infos;
      d.fr.partials = want ? reinterpret_cast<uint4 *>(h->dstate + h->plan.off_partials) : nullptr;
      const int nslots = (int)item_tiles(h, L.compact);
      const int nblk = (nslots + cog::kStatBlock - 1) / cog::kStatBlock;
      d.fr.nslots = nslots;
      d.fr.nframes = it.nframes;
      d.fr.frame0 = h->frame;
      d.b = h->buf;
      d.kp = h->kp;
      d.tile_begin = tb;
      tb += nslots;
      if (want) {
        cog::StatJob sj{};
        sj.partials = d.fr.partials;
        sj.nslots = nslots;
        sj.nframes = it.nframes;
        job_item.push_back((size_t)L.items[q]);
        job_blk.push_back(nblk);
        job_off.push_back(stat_words);
        stat_words += (size_t)it.nframes * nblk * cog::kStat;
        max_blk = std::max(max_blk, nblk);
        max_fr = std::max(max_fr, it.nframes);
        jobs.push_back(sj);
      }
    }
  }
  if (!jobs.empty() && stat_words > b->dstat_cap) {
    if (b->dstat) (void)hipFree(b->dstat);
    b->dstat = nullptr;
    b->dstat_cap = 0;
    hipError_t e = hipMalloc((void **)&b->dstat, stat_words * 4);
    if (e != hipSuccess) return bfail(COG_E_OOM, "statistics allocation failed");
    b->dstat_cap = stat_words;
  }
  for (size_t q = 0; q < jobs.size(); ++q) jobs[q].out = b->dstat + job_off[q];
  char *hjobs = hb + (size_t)kMaxLaunches * b->region_bytes;
  if (!jobs.empty()) std::memcpy(hjobs, jobs.data(), jobs.size() * sizeof(cog::StatJob));

  // uploads: the used prefix of each class region, then the job table
  for (size_t j = 0; j < launches.size(); ++j) {
    const size_t nb = sizeof(cog::TickHead) + launches[j].items.size() * sizeof(cog::TickItem);
    hipError_t e = hipMemcpyAsync(b->ddesc + j * b->region_bytes, hb + j * b->region_bytes, nb,
                                  hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return bhip(e, "descriptor upload");
  }
  char *djobs = b->ddesc + (size_t)kMaxLaunches * b->region_bytes;
  if (!jobs.empty()) {
    hipError_t e = hipMemcpyAsync(djobs, hjobs, jobs.size() * sizeof(cog::StatJob),
                                  hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return bhip(e, "descriptor upload");
  }
  hipError_t e = hipEventRecord(b->hev[cur], b->stream);
  if (e != hipSuccess) return bhip(e, "descriptor staging");
  b->hev_used[cur] = true;
  b->hcur ^= 1;

  // (the legacy default stream cannot be captured)
  bool graph = !launches.empty() && b->stream != nullptr;
  for (const Launch &L : launches) graph = graph && L.graph;
  cog_status s = graph ? run_graph(b, launches) : launch_all(b, launches);
  if (s != COG_OK) return s;

  if (!jobs.empty()) {
    e = cog::launch_stats_table(reinterpret_cast<const cog::StatJob *>(djobs), (int)jobs.size(),
                                max_blk, max_fr, b->stream);
    if (e != hipSuccess) return bhip(e, "statistics launch");
    b->hstat.resize(stat_words);
    e = hipMemcpyAsync(b->hstat.data(), b->dstat, stat_words * 4, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(e, "statistics copy");
    for (size_t q = 0; q < jobs.size(); ++q) {
      const cog_tick_item &it = items[job_item[q]];
      cog_rt::fill_infos(it.ctx, it.ctx->frame, it.nframes, b->hstat.data() + job_off[q], it.infos,
                         job_blk[q]);
    }
  }
  return COG_OK;
}

}  // namespace

extern "C" {

cog_status cog_batch_create(void *hip_stream, int32_t max_items, cog_batch **out) {
  if (!out) return bfail(COG_E_INVALID, "out is NULL");
  *out = nullptr;
  if (max_items < 1 || max_items > kMaxItemsLimit) return bfail(COG_E_INVALID, "max_items must be in [1, 4096]");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return bhip(e, "no HIP device");
  }
  int ncu = 0;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess || ncu < 1) return bhip(e, "device query");
  cog_batch *b = new (std::nothrow) cog_batch();
  if (!b) return bfail(COG_E_OOM, "host allocation failed");
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->device = dev;
  b->ncu = ncu;
  b->max_items = max_items;
  b->region_bytes = align256(sizeof(cog::TickHead) + (size_t)max_items * sizeof(cog::TickItem));
  b->desc_bytes = (size_t)kMaxLaunches * b->region_bytes +
                  align256((size_t)max_items * sizeof(cog::StatJob));
  bool ok = hipMalloc((void **)&b->ddesc, b->desc_bytes) == hipSuccess;
  for (int i = 0; i < 2 && ok; ++i) {
    ok = hipHostMalloc((void **)&b->hdesc[i], b->desc_bytes, hipHostMallocDefault) == hipSuccess;
    if (ok) ok = hipEventCreateWithFlags(&b->hev[i], hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    cog_batch_destroy(b);
    return bfail(COG_E_OOM, "batch allocation failed");
  }
  *out = b;
  return COG_OK;
}

cog_status cog_batch_tick(cog_batch *b, const cog_tick_item *items, int32_t n) {
  std::vector<Launch> launches;
  bool any_infos = false;
  cog_status s = plan_tick(b, items, n, true, launches, any_infos);
  if (s != COG_OK) return s;
  if (launches.empty()) return COG_OK;
  s = execute(b, items, launches, any_infos);
  if (s != COG_OK) return s;
  for (int i = 0; i < n; ++i) items[i].ctx->frame += items[i].nframes;
  return COG_OK;
}

cog_status cog_batch_set_schedule(cog_batch *b, int32_t channels, int32_t K, int32_t dtype,
                                  const cog_schedule *s) {
  if (!b) return bfail(COG_E_INVALID, "batch is NULL");
  const std::string m = check_schedule(s);
  if (!m.empty()) return bfail(COG_E_INVALID, m);
  if ((channels != 1 && channels != 3) || K < 1 || K > 8 || (dtype != COG_U8 && dtype != COG_F32))
    return bfail(COG_E_INVALID, "no such class");
  b->sched[ClassKey{channels, K, dtype == COG_F32 ? 1 : 0, 0}] = *s;
  return COG_OK;
}

cog_status cog_batch_get_schedule(cog_batch *b, int32_t channels, int32_t K, int32_t dtype,
                                  cog_schedule *s) {
  if (!b || !s) return bfail(COG_E_INVALID, "NULL argument");
  if ((channels != 1 && channels != 3) || K < 1 || K > 8 || (dtype != COG_U8 && dtype != COG_F32))
    return bfail(COG_E_INVALID, "no such class");
  auto it = b->sched.find(ClassKey{channels, K, dtype == COG_F32 ? 1 : 0, 0});
  *s = it == b->sched.end() ? default_schedule() : it->second;
  return COG_OK;
}

cog_status cog_batch_autotune(cog_batch *b, const cog_tick_item *items, int32_t n, int32_t reps,
                              cog_schedule *best) {
  if (reps < 1 || reps > 100) return bfail(COG_E_INVALID, "reps must be in [1, 100]");
  std::vector<Launch> launches;
  bool any_infos = false;
  cog_status s = plan_tick(b, items, n, false, launches, any_infos);
  if (s != COG_OK) return s;
  if (launches.empty()) return COG_OK;

  // snapshot of every context's mutable state (everything before the weights)
  std::vector<const cog_ctx *> ctxs;
  for (const Launch &L : launches)
    for (int i : L.items) ctxs.push_back(items[i].ctx);
  std::vector<size_t> off(ctxs.size() + 1, 0);
  for (size_t i = 0; i < ctxs.size(); ++i) off[i + 1] = off[i] + align256(ctxs[i]->plan.off_kdew);
  char *snap = nullptr;
  hipError_t e = hipMalloc((void **)&snap, off.back());
  if (e != hipSuccess) return bfail(COG_E_OOM, "tuning scratch allocation failed");
  auto copy_all = [&](bool save) -> hipError_t {
    for (size_t i = 0; i < ctxs.size(); ++i) {
      char *st = ctxs[i]->dstate;
      hipError_t r = save ? hipMemcpyAsync(snap + off[i], st, ctxs[i]->plan.off_kdew,
                                           hipMemcpyDeviceToDevice, b->stream)
                          : hipMemcpyAsync(st, snap + off[i], ctxs[i]->plan.off_kdew,
                                           hipMemcpyDeviceToDevice, b->stream);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = copy_all(true);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  s = e == hipSuccess ? COG_OK : bhip(e, "tuning setup");

  // candidates: one workgroup per unit, and persistent grids at the
  // occupancy limit and at twice it, units dealt round-robin (the atomic
  // queue is settable but measured far slower, so it is not tried); each
  // with and without the compacting launch for one-frame items
  std::vector<cog_schedule> cand;
  for (int c : {1, 0})
    for (int bpc : {-1, 0, -2})  // -2: twice the occupancy limit
      for (int g : {1, 4, 16}) cand.push_back(cog_schedule{bpc, 0, g, 1, c});

  // one tuning pass per class (a class may have a compacting and a plain
  // launch); the whole tick is timed for every candidate
  std::vector<size_t> firsts;
  std::set<ClassKey> tuned;
  for (size_t j = 0; j < launches.size(); ++j)
    if (tuned.insert(launches[j].key.sched_key()).second) firsts.push_back(j);
  for (size_t fi = 0; fi < firsts.size() && s == COG_OK; ++fi) {
    const size_t j = firsts[fi];
    const ClassKey key = launches[j].key.sched_key();
    float best_ms = 1e30f;
    cog_schedule best_s = default_schedule();
    auto it0 = b->sched.find(key);
    if (it0 != b->sched.end()) best_s = it0->second;
    // the incumbent is timed first; a candidate replaces it only when it is
    // faster by more than the tick-to-tick noise (3 %)
    std::vector<cog_schedule> trial{best_s};
    trial.insert(trial.end(), cand.begin(), cand.end());
    bool first = true;
    for (cog_schedule c : trial) {
      if (c.blocks_per_cu == -2)
        c.blocks_per_cu = std::min(64, 2 * occupancy(b, launches[j].key, launches[j].lp, c.compact != 0));
      b->sched[key] = c;
      std::vector<float> t;
      // one untimed round first (graph capture, cold caches)
      for (int r = -1; r < reps && s == COG_OK; ++r) {
        std::vector<Launch> ls;
        bool dummy = false;
        s = plan_tick(b, items, n, false, ls, dummy);
        if (s != COG_OK) break;
        e = copy_all(false);
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        if (e != hipSuccess) { s = bhip(e, "tuning"); break; }
        s = execute(b, items, ls, false);
        if (s != COG_OK) break;
        e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { s = bhip(e, "tuning"); break; }
        if (r >= 0) t.push_back(ms);
      }
      if (s != COG_OK) break;
      std::sort(t.begin(), t.end());
      const float med = t[t.size() / 2];
      if (first || med < 0.97f * best_ms) {
        best_ms = med;
        best_s = c;
      }
      first = false;
    }
    b->sched[key] = best_s;
    if (fi == 0 && best) *best = best_s;
  }
  // the streams as they were
  if (snap) {
    hipError_t r = copy_all(false);
    if (r == hipSuccess) r = hipStreamSynchronize(b->stream);
    if (r != hipSuccess && s == COG_OK) s = bhip(r, "tuning restore");
    (void)hipFree(snap);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return s;
}

void cog_batch_destroy(cog_batch *b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (GraphEntry &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  for (int i = 0; i < 2; ++i) {
    if (b->hev[i]) (void)hipEventDestroy(b->hev[i]);
    if (b->hdesc[i]) (void)hipHostFree(b->hdesc[i]);
  }
  if (b->ddesc) (void)hipFree(b->ddesc);
  if (b->dstat) (void)hipFree(b->dstat);
  delete b;
}

}  // extern "C"
