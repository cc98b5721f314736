/*
 * cog.h -- C ABI of the MI355X (gfx950) Cascade-of-Gaussians background
 * subtractor (Kiran, Das, Yogamani, "Rejection-Cascade of Gaussians:
 * Real-time adaptive background subtraction framework", arXiv 1705.09339).
 *
 * One context models one video stream.  The problem the calls follow is the
 * paper's: a sequence of frames I_n(x,y) with independent colour channels
 * (§2, "Scene Prior"), a training phase over the first N frames (§2, "Scene
 * Prior" and "Determining Learning Rate Hyper-parameters"), then for every
 * later frame a background/foreground label per pixel produced by the
 * rejection cascade (§2, "Cascade of Gaussians CoG"), with the
 * abrupt-illumination counter of the same paragraph as a side output.
 *
 * Conventions
 *  - Frames are HWC, tightly packed: pixel p = y*width + x, channel c at
 *    byte/element p*channels + c.  u8 frames hold levels 0..255; f32 frames
 *    hold arbitrary values (e.g. latent maps, §3.3) quantised for the prior
 *    over [in_lo, in_hi).
 *  - Masks are width*height bytes, 0 = background, 255 = foreground.
 *  - "on_device" arguments say whether a pointer is HIP device memory (1) or
 *    host memory (0).  Device pointers are used in stream order on the
 *    context's stream and the call returns without waiting; host pointers are
 *    staged through library-owned device buffers and the call waits for the
 *    copies it needs.
 *  - Every call returns a cog_status; no C++ exception crosses the ABI.  A
 *    failed call leaves the context as it was.  cog_last_error() explains the
 *    last failure.
 *  - A context is not thread-safe.  Distinct contexts on distinct streams are
 *    independent.
 */
#ifndef COG_H
#define COG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cog_ctx cog_ctx;

typedef enum {
  COG_OK = 0,
  COG_E_INVALID = -1,     /* bad argument: size, NULL pointer, parameter range */
  COG_E_OOM = -2,         /* device allocation failed or state buffer too small */
  COG_E_STATE = -3,       /* call out of order (step before training, train twice) */
  COG_E_DEVICE = -4,      /* HIP runtime error (no device, launch or copy failure) */
  COG_E_UNSUPPORTED = -5  /* valid but not implemented combination */
} cog_status;

typedef enum { COG_U8 = 0, COG_F32 = 1 } cog_dtype;

/* Cascade stages that may decide a pixel before the mixture (stage_mask). */
enum {
  COG_STAGE_FD = 1u,   /* S0: consistent hypothesis propagation (frame difference) */
  COG_STAGE_RGA = 2u,  /* S1: running Gaussian average */
  COG_STAGE_KDE = 4u,  /* S2: scene-prior confidence */
  COG_STAGE_ALL = 7u,
  COG_STAGE_SAMPLE = 8u /* confidence-based spatio-temporal sampling (off by default) */
};

/* Which kernel family a context runs. */
typedef enum {
  COG_PATH_CASCADE = 0, /* the fused rejection cascade */
  COG_PATH_GMM = 1      /* plain Stauffer-Grimson mixture on every pixel (baseline) */
} cog_path;

/* Parameters (plain data; struct_size = sizeof(cog_params) versions it).
 * Defaults from cog_default_params() are given in brackets. */
typedef struct {
  uint32_t struct_size;
  int32_t width, height;   /* frame size in pixels, each >= 1 */
  int32_t channels;        /* 1 or 3 */
  int32_t dtype;           /* cog_dtype */
  float in_lo, in_hi;      /* f32 input: prior quantisation range [0, 256) */
  int32_t K;               /* mixture components, 1..8 */
  float alpha;             /* mixture learning rate [0.01] */
  float T;                 /* background portion of the weight [0.7] */
  float lambda;            /* match gate in standard deviations [2.5] */
  float var_init;          /* variance of a new component [channels*225] */
  float var_min;           /* variance floor, > 0 [channels*4] */
  uint32_t stage_mask;     /* COG_STAGE_* bits [COG_STAGE_ALL] */
  float tau_fd;            /* S0 tolerance on max_c |x - x'| [0] */
  float lambda_rga;        /* S1 gate in standard deviations [2.5] */
  float alpha_rga;         /* S1 learning rate [alpha] */
  int32_t kde_bins;        /* prior bins per channel; must be 16 [16] */
  float kde_h;             /* prior kernel bandwidth in levels [8] */
  float res_e1, res_e2;    /* residue bin edges (static | oscillating | dynamic) [16, 48] */
  float lambda_m;          /* model-distance scale of the confidence [2*lambda_rga] */
  float conf_thr;          /* S2 accepts background when C >= conf_thr [0.5] */
  float p_null;            /* prior term dropped when P < p_null [0.1] */
  float kappa_alpha;       /* mixture rate alpha*(1 - kappa_alpha*C) [0.5] */
  float illum_frac;        /* illumination flag when n3 > illum_frac*pixels [0.7] */
  int32_t path;            /* cog_path [COG_PATH_CASCADE] */
  int32_t tile_px;         /* cascade pixels per tile: 0 (auto = 64), 64, 128, 256, 512, 1024 */
  /* Confidence-based spatio-temporal sampling (§2 "Confidence based temporal
   * sampling", §3.2), enabled by COG_STAGE_SAMPLE: a pixel decided by frame
   * differencing, or by the running average within samp_lambda standard
   * deviations, on samp_window consecutive evaluated frames has a saturated
   * confidence; a block of 64 consecutive pixels that are all saturated is
   * evaluated only on frames n with (n + block) % samp_period == 0, and on
   * the other frames its labels repeat and nothing adapts.  Cascade path
   * with 64-pixel tiles only. */
  int32_t samp_window;     /* 1..65535 [32] */
  int32_t samp_period;     /* 1..65535 [4] */
  float samp_lambda;       /* >= 0 [lambda_rga] */
} cog_params;

/* Per-frame statistics (the occupancy of the cascade levels, §2 "Cascade of
 * Gaussians CoG" and §3.2, and the illumination counter of §2). */
typedef struct {
  int64_t frame;        /* index of the frame in the stream (training frames count) */
  int64_t n_stage[4];   /* pixels decided at S0, S1, S2; pixels that reached S3 */
  int64_t n3_bg;        /* of those, labelled background by the mixture */
  int64_t n_fg;         /* foreground pixels in the mask */
  int32_t illum_flag;   /* n_stage[3] > illum_frac * pixels */
  int32_t n_skip;       /* pixels of blocks halted by sampling (no level ran) */
} cog_step_info;

/* Fill *p with the defaults above for a w x h stream of c channels.
 * COG_E_INVALID for NULL p. */
cog_status cog_default_params(cog_params *p, int32_t w, int32_t h, int32_t c, int32_t dtype,
                              int32_t K);

/* Device bytes one stream's state needs (model state, prior, previous frame
 * and labels, statistics workspace); for admission against an HBM budget.
 * COG_E_INVALID for bad parameters. */
cog_status cog_state_bytes(const cog_params *p, size_t *bytes);

/* Create a context.  hip_stream: a hipStream_t, or NULL for the default
 * stream.  device_state: NULL to let the library allocate the state with
 * hipMalloc (freed by cog_destroy), or a caller-owned device buffer of at
 * least cog_state_bytes() bytes, 256-byte aligned, that must outlive the
 * context.  Nothing runs on the GPU except the upload of the prior kernel
 * weights.  Errors: COG_E_INVALID (parameters, NULL out, misaligned buffer),
 * COG_E_OOM (allocation failed or state_bytes too small), COG_E_DEVICE. */
cog_status cog_create(const cog_params *p, void *hip_stream, void *device_state,
                      size_t state_bytes, cog_ctx **out);

/* Training phase (§2 "Scene Prior", "Determining Learning Rate
 * Hyper-parameters"): consumes frames 0..n-1 (n x H x W x C, contiguous) and
 * builds, per pixel, the kernel-density prior table, the 3-bin residue
 * histogram and the warmed-up mixture; no masks are produced.  2 <= n <= 65536.
 * COG_E_STATE if already trained. */
cog_status cog_train_prior(cog_ctx *h, const void *frames, int32_t n, int32_t frames_on_device);

/* One frame of the cascade (§2 "Cascade of Gaussians CoG", "Confidence
 * Measure").  mask_out may be NULL.  info may be NULL; when given, the call
 * waits for the frame and fills it.  COG_E_STATE before training. */
cog_status cog_step(cog_ctx *h, const void *frame, int32_t frame_on_device, uint8_t *mask_out,
                    int32_t mask_on_device, cog_step_info *info);

/* n consecutive frames of one stream in one launch (n x H x W x C frames,
 * n x H x W masks).  The result is bit-identical to n cog_step() calls; the
 * per-pixel state stays in registers across the n frames.  infos (n entries)
 * may be NULL; when given, per-tile counter rows (16 bytes per 64 pixels
 * and frame) are reduced on the device and the call waits once at the end.
 * The rows of up to 16..64 frames fit the state (32 MiB); a call over more
 * frames grows a row workspace of the context, up to 1 GiB (hipMalloc on
 * first use, kept until cog_destroy), so that its frames go in one launch
 * (as many launches as the workspace needs; if the allocation fails, in
 * launches of the state's chunk).  1 <= n.  With tile_px = 0 a single frame
 * (n = 1, no sampling) runs the per-frame kernel: 256-pixel tiles whose
 * survivors are compacted into one work list per wave. */
cog_status cog_step_frames(cog_ctx *h, const void *frames, int32_t n, int32_t frames_on_device,
                           uint8_t *masks_out, int32_t masks_on_device, cog_step_info *infos);

/* Return the context to the untrained state (no GPU work, no allocation). */
cog_status cog_reset(cog_ctx *h);

/* Destroy a context; NULL-safe.  Waits for the context's stream. */
void cog_destroy(cog_ctx *h);

/* Canonical, layout-independent state: a 64-byte header {u32 magic 'COG1',
 * u32 version 2, i32 width, height, channels, K, dtype, n_train, i64 frame},
 * then sections each padded to 64 bytes: gmm f32[P][K][C+2] (w, mu[C], var in
 * rank order), rga f32[P][C+1] (mu_r[C], var_r), table u8[P][C][16],
 * cnt u16[P][3], label u8[P] (0/1), prev f32[P][C], sat u16[P] (sampling
 * counters), gkey u32[P][2] (grouping keys) and shared u8[P] (1 where the
 * pixel takes its group's shared variance, cog_group_share): version 3 of the
 * layout.  Version-2 states (without the last section) are imported with no
 * pixel shared, version-1 states (without the last three) also with zero
 * counters and keys.  For checkpoint/resume and tests; synchronous; host
 * buffers only. */
cog_status cog_canonical_bytes(const cog_params *p, size_t *bytes);
cog_status cog_export_state(cog_ctx *h, void *host_dst, size_t bytes);
cog_status cog_import_state(cog_ctx *h, const void *host_src, size_t bytes);

/* Spatio-temporal grouping of the background (§2 "Clustering Similar
 * Background - Spatio-Temporal Grouping"), on a trained cascade context.
 * Per pixel the training warm-up recorded the temporal variance of the
 * dominant component's adapted variance and of its weight (the diagonal of
 * the paper's Cov(V), Cov(R)), as integer keys (binary32 pattern >> 16).
 * Integer k-means with 3 clusters (initial centres: min, mean, max of each
 * key; nearest centre, lowest index on ties; centres at the floor of their
 * members' mean; until no change, at most 32 passes) groups the pixels; a
 * pixel stays in its cluster when both keys lie within one standard
 * deviation of the cluster's member mean (eq. 3, closed interval).
 * map_out (P bytes, device or host, may be NULL): cluster 0..2, 255 for an
 * ungrouped pixel.  info may be NULL.  Synchronous; uses temporary device
 * memory.  COG_E_STATE before training; COG_E_UNSUPPORTED on the baseline
 * path. */
typedef struct {
  int64_t count;        /* pixels assigned to the cluster */
  int64_t grouped;      /* of those, inside the one-sigma band */
  int64_t center[2];    /* final centre (keys) */
  double mean[2], sd[2];
} cog_group_stats;
typedef struct {
  int32_t iterations;
  int32_t reserved;
  cog_group_stats group[3];
} cog_group_info;
cog_status cog_group_background(cog_ctx *h, uint8_t *map_out, int32_t map_on_device,
                                cog_group_info *info);

/* One shared parameter set per group (§2 "Clustering Similar Background",
 * the last item of its list and eq. 3): the pixels of each group take one
 * variance for their running Gaussian average (the first, dominant cascade
 * level), fitted once as the mean of the members' current variances, and no
 * longer adapt it; their means keep adapting per pixel.  The mean is exact
 * on a fixed-point grid: each member's variance rounded to a multiple of
 * 2^-16 (binary64 rint, ties to even), the integers summed, one binary64
 * division, then binary32, held at var_min or above.
 * map (P bytes, device when map_on_device != 0, else host): group 0..2 per
 * pixel, 255 for a pixel outside every group, e.g. the map written by
 * cog_group_background; NULL ungroups every pixel (each then adapts its
 * variance again from the value it holds).  Pixels outside the groups keep
 * their own variance.  gvar_out (3 floats, may be NULL): the shared
 * variances, 0 for an empty group.  Training clears the sharing.  The flag
 * travels in the canonical state's shared section.  Synchronous; uses
 * temporary device memory.  COG_E_STATE before training, COG_E_UNSUPPORTED
 * on the baseline path, COG_E_INVALID for a map value other than 0..2 and
 * 255 or a member variance of 2^37 or more (nothing is changed then). */
cog_status cog_group_share(cog_ctx *h, const uint8_t *map, int32_t map_on_device,
                           float *gvar_out);

/* The same grouping without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Its scratch (assignment and map planes, per-block sums)
 * is a static device array of about 20 MiB that every GPU the library runs on
 * holds until the process ends; its address is looked up per GPU by
 * cog_create.  Streams of at most COG_NOALLOC_MAX_PIXELS pixels, else
 * COG_E_INVALID; COG_E_DEVICE if the scratch could not be located.  Every
 * call on one GPU shares that GPU's scratch and leaves its contents behind
 * (each call initialises what it reads): calls that overlap on one GPU, from
 * several host threads or on several streams, race, and the caller must
 * serialise them.  Arguments, results and errors otherwise as
 * cog_group_background; synchronous. */
#define COG_NOALLOC_MAX_PIXELS (1 << 23)
cog_status cog_group_background_noalloc(cog_ctx *h, uint8_t *map_out, int32_t map_on_device,
                                        cog_group_info *info);

/* Integer prior kernel weights W[b][v] (16 x 256, row-major) for bandwidth h,
 * as used by the training kernel; host-only, needs no GPU. */
cog_status cog_kde_weights(float h, uint16_t *out);

/* Message of the last failure on h (or of the calling thread if h is NULL). */
const char *cog_last_error(const cog_ctx *h);

/* ---- Batched tick -----------------------------------------------------------
 * Many streams advanced together: every pixel of every stream is independent
 * (§2, "Cascade of Gaussians CoG": the cascade is a per-pixel decision
 * list), so the 64-pixel tiles of all streams of one tick form a single work
 * list.  A tick runs one persistent launch per class of streams (channels,
 * K, input type), replayed from a captured hipGraph, on the batch's stream.
 * For every item the result (masks, statistics, state) is bit-identical to
 * cog_step_frames() on that stream alone.
 *
 * Ownership: the batch owns its descriptor buffers, graphs and tuning
 * scratch; it borrows the contexts and the frame/mask buffers of a tick until
 * the tick's work on the stream completes.  A context may take part in ticks
 * of one batch and in one-stream calls, in any order, as long as it was
 * created on the batch's stream. */
typedef struct cog_batch cog_batch;

/* One stream's work in a tick. */
typedef struct {
  cog_ctx *ctx;           /* trained context, cascade path, 64-pixel tiles (tile_px 0 or 64) */
  const void *frames;     /* device: nframes x H x W x C, contiguous */
  uint8_t *masks;         /* device: nframes x H x W, or NULL */
  int32_t nframes;        /* >= 0 (0: the item is skipped); with infos at most the
                             stream's statistics chunk: 16..64 frames, as many as
                             fit 32 MiB of 16-byte per-tile rows (64 at 1920x1080) */
  int32_t reserved;       /* must be 0 */
  cog_step_info *infos;   /* host array of nframes entries, or NULL */
} cog_tick_item;

/* How a class's tiles are spread over the GPU. */
typedef struct {
  int32_t blocks_per_cu;  /* persistent workgroups per compute unit; 0: the occupancy limit;
                             -1: no persistence, one workgroup per schedule unit */
  int32_t dynamic;        /* 0: units dealt round-robin; 1: taken from an atomic counter */
  int32_t group;          /* tiles per schedule unit, 1..1024 */
  int32_t use_graph;      /* 1: replay a captured hipGraph; 0: launch directly */
  int32_t compact;        /* 1: the class's items that advance by one frame (no
                             sampling) run in a launch of their own with 256-pixel
                             tiles whose S1 survivors are compacted into one work
                             list per wave (as cog_step with tile_px 0); 0: every
                             item runs in 64-pixel one-pixel-per-lane tiles */
} cog_schedule;

/* Create a batch on hip_stream (NULL: default stream) for up to max_items
 * items per tick (1..4096).  Errors: COG_E_INVALID, COG_E_OOM, COG_E_DEVICE. */
cog_status cog_batch_create(void *hip_stream, int32_t max_items, cog_batch **out);

/* Advance every item's stream by its nframes frames.  Stream-ordered and
 * non-blocking unless an item has infos (then the call waits and fills
 * them).  Errors (nothing runs): COG_E_INVALID (NULL or duplicate context,
 * context on another stream, bad counts, more than 8 classes),
 * COG_E_STATE (untrained context), COG_E_UNSUPPORTED (baseline path or
 * tiles other than 64 pixels), COG_E_DEVICE. */
cog_status cog_batch_tick(cog_batch *b, const cog_tick_item *items, int32_t n);

/* Time candidate schedules on this tick's work (reps ticks each, median)
 * and keep, per class, the current schedule unless a candidate is more than
 * 3 % faster (then the fastest).  Candidates: one workgroup per schedule
 * unit, or persistent grids at the occupancy limit and at twice it; units of
 * 1, 4 or 16 tiles; with and without the compacting launch for one-frame
 * items (18 in all).  Every context's state is restored after each
 * trial, so the streams are left as they were; the masks of the items are
 * written (with the tick's result) and no infos are filled.  best (may be
 * NULL) receives the schedule kept for the first item's class.  Needs
 * device scratch equal to the items' state bytes.  Errors as for a tick. */
cog_status cog_batch_autotune(cog_batch *b, const cog_tick_item *items, int32_t n, int32_t reps,
                              cog_schedule *best);

/* Set or read the schedule of one class (channels, K, dtype).  Classes
 * without a set schedule use {-1, 0, 4, 1}.  COG_E_INVALID for bad values. */
cog_status cog_batch_set_schedule(cog_batch *b, int32_t channels, int32_t K, int32_t dtype,
                                  const cog_schedule *s);
cog_status cog_batch_get_schedule(cog_batch *b, int32_t channels, int32_t K, int32_t dtype,
                                  cog_schedule *s);

/* Destroy a batch; NULL-safe.  Waits for its stream.  The contexts stay. */
void cog_batch_destroy(cog_batch *b);

/* ---- Serving loop -------------------------------------------------------------
 * A request loop over many camera streams (the paper's real-time setting,
 * §1 and §3.2): frames are submitted as they arrive; a scheduler thread
 * gathers, whenever fewer than `depth` ticks are in flight, the oldest
 * pending submission of every stream into one batched tick (continuous
 * batching: frames that arrive while a tick runs join the next one), so the
 * work of different requests overlaps on the device.  Every stream's state
 * stays resident in device memory from open to close; the HBM budget is
 * reserved once at creation and a stream is admitted only if its state fits
 * in a free range of it (ranges of closed streams are reused, neighbours
 * merged), so serving never allocates or frees device memory.  A new
 * stream's training runs on the server's stream in slices of pixels that
 * alternate with the ticks (a tick waits for at most one slice), and its
 * frames join the first tick after the last slice.  Each stream's masks and
 * state are bit-identical to the same frames run alone through
 * cog_step_frames.
 *
 * Threading: every call may come from any thread; calls are serialised by
 * the server.  Frames and masks are device buffers owned by the caller and
 * must stay valid until the frame's completion is reported. */
typedef struct cog_server cog_server;

typedef struct {
  int32_t stream_id;
  int32_t nframes;      /* frames of the submission */
  int64_t tag;          /* the caller's tag from cog_server_submit */
  double t_submit_us;   /* host clock at submission, microseconds since cog_server_create */
  double t_done_us;     /* host clock when the tick was seen complete */
  int32_t status;       /* COG_OK, or the error that failed the tick */
  int32_t reserved;
} cog_completion;

typedef struct {
  int64_t ticks;            /* batched ticks issued */
  int64_t frames;           /* frames completed */
  int64_t pixel_frames;     /* pixels x frames completed */
  int64_t streams_open;
  int64_t streams_admitted; /* cog_server_open successes */
  int64_t streams_rejected; /* cog_server_open refusals for lack of budget */
  int64_t bytes_budget;     /* device bytes the server may hold for stream state */
  int64_t bytes_allocated;  /* reserved at creation (the budget, rounded to 256 B) */
  int64_t bytes_in_use;     /* open streams' state */
  int64_t bytes_largest_free; /* largest contiguous free range of the reservation */
  int64_t pending;          /* submissions not yet issued */
  int64_t in_flight;        /* ticks issued and not yet complete */
} cog_server_stats;

/* Create a server on hip_stream (NULL: the server creates its own stream)
 * reserving hbm_budget bytes of device memory for stream state, for at most
 * max_streams streams (1..4096); depth = ticks in flight (1..8).  Errors:
 * COG_E_INVALID, COG_E_OOM (the budget cannot be reserved), COG_E_DEVICE. */
cog_status cog_server_create(void *hip_stream, size_t hbm_budget, int32_t max_streams,
                             int32_t depth, cog_server **out);

/* Admit a stream: reserve its state within the budget, create its context
 * (parameters as for cog_create; cascade path, 64-pixel tiles) and run its
 * training on n_train device frames.  *id receives the stream's id.  The
 * training is issued later by the scheduler, in slices between ticks, and
 * the call returns at once: train_frames must stay valid until the training
 * has ended, that is until the stream's first completion is reported or
 * until cog_server_drain of the stream (or of all streams) returns.
 * COG_E_OOM when the state does not fit the budget or max_streams streams
 * are open; COG_E_INVALID for n_train outside 2..65536; other errors as for
 * cog_create and cog_train_prior. */
cog_status cog_server_open(cog_server *s, const cog_params *p, const void *train_frames,
                           int32_t n_train, int32_t *id);

/* Queue nframes consecutive device frames of stream id (masks: nframes x H x W
 * device bytes, or NULL); returns at once.  COG_E_INVALID for an unknown or
 * closing stream or bad counts (1..64 frames); COG_E_DEVICE if the server
 * has failed. */
cog_status cog_server_submit(cog_server *s, int32_t id, const void *frames, int32_t nframes,
                             uint8_t *masks, int64_t tag);

/* Close stream id.  Its queued frames still complete, after the rest of its
 * training, and then its state range returns to the reservation.  With
 * nothing queued, the training slices not yet issued are dropped; the call
 * waits for those in flight and returns the range at once.  COG_E_INVALID
 * for an unknown or already closing id. */
cog_status cog_server_close(cog_server *s, int32_t id);

/* Move up to max completions (oldest first) to out; *n receives the count.
 * Waits up to wait_us microseconds when none is ready. */
cog_status cog_server_poll(cog_server *s, cog_completion *out, int32_t max, int32_t *n,
                           int64_t wait_us);

/* Wait until every submitted frame (of stream id, or of all streams if
 * id < 0) has completed and the training of those streams has ended. */
cog_status cog_server_drain(cog_server *s, int32_t id);

/* Canonical state of stream id (see cog_export_state), after its submitted
 * frames complete. */
cog_status cog_server_export(cog_server *s, int32_t id, void *host_dst, size_t bytes);

cog_status cog_server_stats_get(cog_server *s, cog_server_stats *out);

/* Stop the scheduler, wait for the device, free everything; NULL-safe. */
void cog_server_destroy(cog_server *s);

#ifdef __cplusplus
}
#endif
#endif /* COG_H */
