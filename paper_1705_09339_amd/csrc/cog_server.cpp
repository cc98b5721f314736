// Host runtime of the serving loop (include/cog.h, "Serving loop").
//
// Two threads per server: a scheduler that issues ticks and a completer that
// waits for them.  The HIP work of a server's streams (training, ticks,
// exports) is enqueued on the server's stream while holding the server
// mutex, so it is ordered; the completer releases the mutex while it waits
// for the oldest tick in flight.  A new stream's training runs there too, in
// slices of kSlicePixels pixels issued between ticks: a tick waits for at
// most one slice, where one whole-stream training launch (several
// milliseconds at 3840x2160) would hold every tick behind it or compete with
// it for the compute units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "cog.h"
#include "cog_ctx.h"

namespace {

struct Submission {
  const void *frames;
  uint8_t *masks;
  int32_t n;
  int64_t tag;
  double t_submit;
};

struct SStream {
  cog_ctx *ctx = nullptr;
  char *state = nullptr;
  size_t bytes = 0;
  int64_t pixels = 0;
  bool closing = false;
  int in_flight = 0;         // submissions and training slices issued and not complete
  int slices_in_flight = 0;  // of those, training slices
  // training still to issue: slices cover the pixels [train_next, pixels)
  bool training = false;
  const void *train_frames = nullptr;
  int32_t n_train = 0;
  int64_t train_next = 0;
  std::deque<Submission> q;
};

// Pixels per training slice: about 0.2 ms of a 1920x1080 K=5 stream's
// training (a multiple of 128, the training workgroup).
constexpr int64_t kSlicePixels = 1 << 18;

struct Issued {
  int32_t id;
  int32_t n;
  int64_t tag;
  double t_submit;
  int64_t pixel_frames;
};

struct Tick {
  hipEvent_t ev = nullptr;
  std::vector<Issued> work;
  int32_t slice_of = -1;  // a training slice of this stream (no work)
  cog_status status = COG_OK;
};

using Clock = std::chrono::steady_clock;

// The budget is reserved as one device allocation at creation; stream states
// are carved out of it (best fit, neighbours coalesced on release), so
// admissions and departures never call hipMalloc or hipFree, which would
// wait for the whole device.
struct Arena {
  char *base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes

  bool take(size_t n, size_t *off) {
    auto best = free_.end();
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n && (best == free_.end() || it->second < best->second)) best = it;
    if (best == free_.end()) return false;
    *off = best->first;
    const size_t rest = best->second - n;
    free_.erase(best);
    if (rest) free_[*off + n] = rest;
    return true;
  }

  void give(size_t off, size_t n) {
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + n == nx->first) {
      n += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += n;
        return;
      }
    }
    free_[off] = n;
  }

  size_t largest() const {
    size_t m = 0;
    for (auto &kv : free_) m = std::max(m, kv.second);
    return m;
  }
};

}  // namespace

struct cog_server {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t train_stream = nullptr;  // admissions upload their weights here
  std::deque<int32_t> train_q;         // streams with training slices to issue, in order
  int device = 0;
  size_t budget = 0, in_use = 0;
  int opening = 0;  // admissions reserved and not yet registered
  int32_t max_streams = 0;
  int depth = 2;
  cog_batch *batch = nullptr;
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::map<int32_t, SStream> streams;
  int32_t next_id = 0;
  Arena arena;
  std::deque<Tick> in_flight;
  std::vector<hipEvent_t> spare_events;
  std::deque<cog_completion> done;
  std::condition_variable cv_flight;
  std::thread scheduler, completer;
  bool stop = false;
  bool sched_done = false;
  cog_status sticky = COG_OK;
  std::string sticky_msg;
  int64_t ticks = 0, frames = 0, pixel_frames = 0, admitted = 0, rejected = 0;
};

namespace {

using cog_rt::fail;

cog_status sfail(cog_status s, const std::string &msg) { return fail(nullptr, s, msg); }

double now_us(const cog_server *s) {
  return std::chrono::duration<double, std::micro>(Clock::now() - s->t0).count();
}

// Frees a finished stream's context (its state returns to the arena).
// The context owns no device memory here and no work refers to it, so
// nothing needs to wait.
void finalize(cog_server *s, int32_t id) {
  auto it = s->streams.find(id);
  if (it == s->streams.end()) return;
  SStream &st = it->second;
  if (st.ctx->own_state || st.ctx->stage_in || st.ctx->stage_mask)
    cog_destroy(st.ctx);
  else
    delete st.ctx;
  s->arena.give((size_t)(st.state - s->arena.base), st.bytes);
  s->in_use -= st.bytes;
  s->streams.erase(it);
}

// Completion of the oldest tick (called with the mutex held, after its
// event has completed or failed).
void retire_front(cog_server *s, cog_status st) {
  Tick t = std::move(s->in_flight.front());
  s->in_flight.pop_front();
  const double td = now_us(s);
  if (st == COG_OK) st = t.status;
  for (const Issued &w : t.work) {
    cog_completion c{};
    c.stream_id = w.id;
    c.nframes = w.n;
    c.tag = w.tag;
    c.t_submit_us = w.t_submit;
    c.t_done_us = td;
    c.status = st;
    s->done.push_back(c);
    if (st == COG_OK) {
      s->frames += w.n;
      s->pixel_frames += w.pixel_frames;
    }
    auto it = s->streams.find(w.id);
    if (it != s->streams.end()) {
      SStream &ss = it->second;
      ss.in_flight -= 1;
      if (ss.closing && ss.q.empty() && ss.in_flight == 0 && !ss.training) finalize(s, w.id);
    }
  }
  if (t.slice_of >= 0) {
    auto it = s->streams.find(t.slice_of);
    if (it != s->streams.end()) {
      SStream &ss = it->second;
      ss.in_flight -= 1;
      ss.slices_in_flight -= 1;
      if (ss.closing && ss.q.empty() && ss.in_flight == 0 && !ss.training) finalize(s, t.slice_of);
    }
  }
  if (t.ev) s->spare_events.push_back(t.ev);
  s->cv_done.notify_all();
}

// Whether every slice of a stream's training has been issued: its frames
// may join the next tick, which the server's stream runs after them.
bool trained(const SStream &st) { return !st.training; }

// An event recorded on the server's stream for a tick or a slice.
hipEvent_t take_event(cog_server *s) {
  hipEvent_t ev = nullptr;
  if (s->spare_events.empty()) {
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      s->sticky = COG_E_DEVICE;
      s->sticky_msg = "event creation failed";
      return nullptr;
    }
  } else {
    ev = s->spare_events.back();
    s->spare_events.pop_back();
  }
  return ev;
}

// Issues the next training slice of the oldest stream still training.
bool issue_slice(cog_server *s) {
  while (!s->train_q.empty()) {
    const int32_t id = s->train_q.front();
    auto it = s->streams.find(id);
    if (it == s->streams.end() || !it->second.training) {
      s->train_q.pop_front();
      continue;
    }
    SStream &st = it->second;
    if (st.closing && st.q.empty()) {
      // closed with nothing queued: the rest of its training is not needed
      st.training = false;
      s->train_q.pop_front();
      if (st.in_flight == 0) finalize(s, id);
      continue;
    }
    const int64_t p1 = std::min(st.pixels, st.train_next + kSlicePixels);
    Tick t;
    t.slice_of = id;
    t.status = cog_rt::train_range(st.ctx, st.train_frames, st.n_train, st.train_next, p1, s->stream);
    if (t.status != COG_OK) {
      s->sticky = t.status;
      s->sticky_msg = cog_last_error(st.ctx);
    }
    st.train_next = p1;
    st.in_flight += 1;
    st.slices_in_flight += 1;
    if (p1 == st.pixels) {
      cog_rt::train_finish(st.ctx, st.n_train);
      st.training = false;
      st.train_frames = nullptr;
      s->train_q.pop_front();
    }
    t.ev = take_event(s);
    if (t.ev && hipEventRecord(t.ev, s->stream) != hipSuccess) t.status = COG_E_DEVICE;
    s->in_flight.push_back(std::move(t));
    return true;
  }
  return false;
}

// Gathers the oldest submission of every stream into one tick and issues it.
bool issue_tick(cog_server *s) {
  std::vector<cog_tick_item> items;
  Tick t;
  for (auto &kv : s->streams) {
    SStream &st = kv.second;
    if (st.q.empty() || !trained(st)) continue;
    const Submission &sub = st.q.front();
    cog_tick_item it{};
    it.ctx = st.ctx;
    it.frames = sub.frames;
    it.masks = sub.masks;
    it.nframes = sub.n;
    items.push_back(it);
    t.work.push_back(Issued{kv.first, sub.n, sub.tag, sub.t_submit, st.pixels * sub.n});
  }
  if (items.empty()) return false;
  cog_status rc = cog_batch_tick(s->batch, items.data(), (int32_t)items.size());
  if (rc != COG_OK) {
    s->sticky = rc;
    s->sticky_msg = cog_last_error(nullptr);
  }
  for (const Issued &w : t.work) {
    SStream &st = s->streams[w.id];
    st.q.pop_front();
    st.in_flight += 1;
  }
  t.ev = take_event(s);
  t.status = rc;
  if (t.ev && hipEventRecord(t.ev, s->stream) != hipSuccess) t.status = COG_E_DEVICE;
  s->in_flight.push_back(std::move(t));
  s->ticks += 1;
  return true;
}

// Completes the queued submissions of a failed server with its failure (and
// drops the training still to issue).
void fail_pending(cog_server *s) {
  s->train_q.clear();
  for (auto &kv : s->streams) {
    kv.second.training = false;
    while (!kv.second.q.empty()) {
      const Submission &sub = kv.second.q.front();
      cog_completion c{};
      c.stream_id = kv.first;
      c.nframes = sub.n;
      c.tag = sub.tag;
      c.t_submit_us = sub.t_submit;
      c.t_done_us = now_us(s);
      c.status = s->sticky;
      s->done.push_back(c);
      kv.second.q.pop_front();
    }
  }
  s->cv_done.notify_all();
}

bool any_pending(const cog_server *s) {
  for (auto &kv : s->streams)
    if (!kv.second.q.empty()) return true;
  return false;
}

// Scheduler: whenever fewer than depth ticks and slices are in flight, issues
// a tick of what is queued or the next training slice, alternating between
// the two while both wait.
void scheduler_main(cog_server *s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  bool slice_next = false;
  while (true) {
    const bool pending = any_pending(s);
    const bool train = !s->train_q.empty();
    if (s->stop && !pending && !train) break;
    if ((pending || train) && s->sticky != COG_OK) {
      fail_pending(s);
      continue;
    }
    if ((pending || train) && (int)s->in_flight.size() < s->depth) {
      bool issued = false;
      if (train && (slice_next || !pending)) issued = issue_slice(s);
      if (!issued && pending) issued = issue_tick(s);
      if (issued) {
        slice_next = s->in_flight.back().slice_of < 0;
      } else if (train) {
        // everything queued waits for training
        issued = issue_slice(s);
        slice_next = false;
      }
      if (issued) {
        s->cv_flight.notify_one();
        continue;
      }
      // nothing issued because the training queue held only streams closed
      // before their slices ran, which issue_slice has dropped: test the
      // loop's conditions again, since a stop may already be waiting and no
      // completion would wake this thread
      if (train && s->train_q.empty()) continue;
    }
    s->cv_work.wait(lk);
  }
  s->sched_done = true;
  s->cv_flight.notify_one();
}

// Completer: waits for the oldest tick in flight (without the mutex) and
// reports its submissions.
void completer_main(cog_server *s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    if (s->in_flight.empty()) {
      if (s->sched_done) break;
      s->cv_flight.wait(lk);
      continue;
    }
    hipEvent_t ev = s->in_flight.front().ev;
    hipError_t e = hipErrorInvalidValue;
    if (ev) {
      lk.unlock();
      e = hipEventSynchronize(ev);
      lk.lock();
    }
    retire_front(s, e == hipSuccess ? COG_OK : COG_E_DEVICE);
    s->cv_work.notify_one();  // a pipeline slot is free
  }
}

bool idle(cog_server *s, int32_t id) {
  if (id >= 0) {
    auto it = s->streams.find(id);
    return it == s->streams.end() ||
           (it->second.q.empty() && it->second.in_flight == 0 && !it->second.training);
  }
  for (auto &kv : s->streams)
    if (!kv.second.q.empty() || kv.second.in_flight || kv.second.training) return false;
  return s->in_flight.empty();
}

}  // namespace

extern "C" {

cog_status cog_server_create(void *hip_stream, size_t hbm_budget, int32_t max_streams,
                             int32_t depth, cog_server **out) {
  if (!out) return sfail(COG_E_INVALID, "out is NULL");
  *out = nullptr;
  if (max_streams < 1 || max_streams > 4096) return sfail(COG_E_INVALID, "max_streams must be in [1, 4096]");
  if (depth < 1 || depth > 8) return sfail(COG_E_INVALID, "depth must be in [1, 8]");
  if (hbm_budget == 0) return sfail(COG_E_INVALID, "hbm_budget must be positive");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return sfail(COG_E_DEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
  }
  cog_server *s = new (std::nothrow) cog_server();
  if (!s) return sfail(COG_E_OOM, "host allocation failed");
  s->device = dev;
  s->budget = hbm_budget;
  s->max_streams = max_streams;
  s->depth = depth;
  s->t0 = Clock::now();
  if (hip_stream) {
    s->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete s;
      return sfail(COG_E_DEVICE, "stream creation failed");
    }
    s->own_stream = true;
  }
  s->budget = (hbm_budget + 255) & ~(size_t)255;
  if (hipMalloc((void **)&s->arena.base, s->budget) != hipSuccess) {
    (void)hipGetLastError();
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return sfail(COG_E_OOM, "the HBM budget could not be reserved");
  }
  s->arena.size = s->budget;
  s->arena.free_[0] = s->budget;
  cog_status rc = cog_batch_create(s->stream, max_streams, &s->batch);
  if (rc == COG_OK && hipStreamCreateWithFlags(&s->train_stream, hipStreamNonBlocking) != hipSuccess) {
    cog_batch_destroy(s->batch);
    rc = sfail(COG_E_DEVICE, "stream creation failed");
  }
  if (rc != COG_OK) {
    (void)hipFree(s->arena.base);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return rc;
  }
  try {
    s->completer = std::thread(completer_main, s);
    s->scheduler = std::thread(scheduler_main, s);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
      s->sched_done = true;
    }
    s->cv_flight.notify_all();
    if (s->completer.joinable()) s->completer.join();
    cog_batch_destroy(s->batch);
    (void)hipStreamDestroy(s->train_stream);
    (void)hipFree(s->arena.base);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return sfail(COG_E_OOM, "thread creation failed");
  }
  *out = s;
  return COG_OK;
}

cog_status cog_server_open(cog_server *s, const cog_params *p, const void *train_frames,
                           int32_t n_train, int32_t *id) {
  if (!s || !p || !id) return sfail(COG_E_INVALID, "NULL argument");
  if (!train_frames) return sfail(COG_E_INVALID, "train_frames is NULL");
  if (p->struct_size == sizeof(cog_params) && p->path != COG_PATH_CASCADE)
    return sfail(COG_E_UNSUPPORTED, "served streams run the cascade path");
  if (p->struct_size == sizeof(cog_params) && p->tile_px != 0 && p->tile_px != 64)
    return sfail(COG_E_UNSUPPORTED, "served streams use 64-pixel tiles");
  size_t bytes = 0;
  cog_status rc = cog_state_bytes(p, &bytes);
  if (rc != COG_OK) return rc;
  bytes = (bytes + 255) & ~(size_t)255;
  char *buf = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->sticky != COG_OK) return sfail(s->sticky, "server failed: " + s->sticky_msg);
    if ((int32_t)s->streams.size() + s->opening >= s->max_streams) {
      s->rejected += 1;
      return sfail(COG_E_OOM, "the server holds max_streams streams");
    }
    size_t off = 0;
    if (!s->arena.take(bytes, &off)) {
      s->rejected += 1;
      return sfail(COG_E_OOM, "stream state does not fit the HBM budget");
    }
    buf = s->arena.base + off;
    s->in_use += bytes;
    s->opening += 1;
  }
  // Built without the server lock, so ticks keep flowing: the context is
  // created on the side stream (the weight upload waits only for that
  // stream); its training is issued by the scheduler in slices between ticks,
  // and its frames join the first tick after the last slice.
  cog_ctx *ctx = nullptr;
  if (n_train < 2 || n_train > 65536) rc = sfail(COG_E_INVALID, "training needs 2 <= n <= 65536 frames");
  else rc = cog_create(p, s->train_stream, buf, bytes, &ctx);
  std::lock_guard<std::mutex> lk(s->mu);
  s->opening -= 1;
  if (rc != COG_OK) {
    std::string msg = ctx ? cog_last_error(ctx) : cog_last_error(nullptr);
    if (ctx) delete ctx;
    s->arena.give((size_t)(buf - s->arena.base), bytes);
    s->in_use -= bytes;
    return sfail(rc, msg);
  }
  ctx->stream = s->stream;
  const int32_t nid = s->next_id++;
  SStream &st = s->streams[nid];
  st.ctx = ctx;
  st.state = buf;
  st.bytes = bytes;
  st.pixels = (int64_t)p->width * p->height;
  st.training = true;
  st.train_frames = train_frames;
  st.n_train = n_train;
  st.train_next = 0;
  s->train_q.push_back(nid);
  s->admitted += 1;
  s->cv_work.notify_one();
  *id = nid;
  return COG_OK;
}

cog_status cog_server_submit(cog_server *s, int32_t id, const void *frames, int32_t nframes,
                             uint8_t *masks, int64_t tag) {
  if (!s) return sfail(COG_E_INVALID, "server is NULL");
  if (!frames) return sfail(COG_E_INVALID, "frames is NULL");
  if (nframes < 1 || nframes > 64) return sfail(COG_E_INVALID, "nframes must be in [1, 64]");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->sticky != COG_OK) return sfail(s->sticky, "server failed: " + s->sticky_msg);
    auto it = s->streams.find(id);
    if (it == s->streams.end() || it->second.closing) return sfail(COG_E_INVALID, "no such open stream");
    it->second.q.push_back(Submission{frames, masks, nframes, tag, now_us(s)});
  }
  s->cv_work.notify_one();
  return COG_OK;
}

cog_status cog_server_close(cog_server *s, int32_t id) {
  if (!s) return sfail(COG_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->streams.find(id);
  if (it == s->streams.end() || it->second.closing) return sfail(COG_E_INVALID, "no such open stream");
  SStream &st = it->second;
  st.closing = true;
  if (st.q.empty()) {
    // nothing of the stream remains to run: the rest of its training is not
    // needed, and once its slices in flight have ended (they are waited for
    // here) its range returns at once
    st.training = false;
    if (st.in_flight == st.slices_in_flight) {
      for (const Tick &t : s->in_flight)
        if (t.slice_of == id && t.ev) (void)hipEventSynchronize(t.ev);
      finalize(s, id);
    }
  }
  return COG_OK;
}

cog_status cog_server_poll(cog_server *s, cog_completion *out, int32_t max, int32_t *n,
                           int64_t wait_us) {
  if (!s || !n || (max > 0 && !out)) return sfail(COG_E_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [s] { return !s->done.empty(); });
  int k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n = k;
  return COG_OK;
}

cog_status cog_server_drain(cog_server *s, int32_t id) {
  if (!s) return sfail(COG_E_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_work.notify_one();
  s->cv_done.wait(lk, [s, id] { return idle(s, id) || s->sticky != COG_OK; });
  if (s->sticky != COG_OK) return sfail(s->sticky, "server failed: " + s->sticky_msg);
  return COG_OK;
}

cog_status cog_server_export(cog_server *s, int32_t id, void *host_dst, size_t bytes) {
  if (!s) return sfail(COG_E_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [s, id] { return idle(s, id) || s->sticky != COG_OK; });
  if (s->sticky != COG_OK) return sfail(s->sticky, "server failed: " + s->sticky_msg);
  auto it = s->streams.find(id);
  if (it == s->streams.end()) return sfail(COG_E_INVALID, "no such open stream");
  return cog_export_state(it->second.ctx, host_dst, bytes);
}

cog_status cog_server_stats_get(cog_server *s, cog_server_stats *out) {
  if (!s || !out) return sfail(COG_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->ticks = s->ticks;
  out->frames = s->frames;
  out->pixel_frames = s->pixel_frames;
  out->streams_open = (int64_t)s->streams.size();
  out->streams_admitted = s->admitted;
  out->streams_rejected = s->rejected;
  out->bytes_budget = (int64_t)s->budget;
  out->bytes_allocated = (int64_t)s->arena.size;
  out->bytes_in_use = (int64_t)s->in_use;
  out->bytes_largest_free = (int64_t)s->arena.largest();
  int64_t pend = 0;
  for (auto &kv : s->streams) pend += (int64_t)kv.second.q.size();
  out->pending = pend;
  out->in_flight = (int64_t)s->in_flight.size();
  return COG_OK;
}

void cog_server_destroy(cog_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->scheduler.joinable()) s->scheduler.join();
  if (s->completer.joinable()) s->completer.join();
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamSynchronize(s->train_stream);
  std::vector<int32_t> ids;
  for (auto &kv : s->streams) ids.push_back(kv.first);
  for (int32_t id : ids) finalize(s, id);
  (void)hipFree(s->arena.base);
  for (hipEvent_t e : s->spare_events)
    if (e) (void)hipEventDestroy(e);
  cog_batch_destroy(s->batch);
  (void)hipStreamDestroy(s->train_stream);
  if (s->own_stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
