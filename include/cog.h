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
  COG_STAGE_ALL = 7u
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
} cog_params;

/* Per-frame statistics (the occupancy of the cascade levels, §2 "Cascade of
 * Gaussians CoG" and §3.2, and the illumination counter of §2). */
typedef struct {
  int64_t frame;        /* index of the frame in the stream (training frames count) */
  int64_t n_stage[4];   /* pixels decided at S0, S1, S2; pixels that reached S3 */
  int64_t n3_bg;        /* of those, labelled background by the mixture */
  int64_t n_fg;         /* foreground pixels in the mask */
  int32_t illum_flag;   /* n_stage[3] > illum_frac * pixels */
  int32_t reserved;
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
 * may be NULL; when given the call waits.  1 <= n. */
cog_status cog_step_frames(cog_ctx *h, const void *frames, int32_t n, int32_t frames_on_device,
                           uint8_t *masks_out, int32_t masks_on_device, cog_step_info *infos);

/* Return the context to the untrained state (no GPU work, no allocation). */
cog_status cog_reset(cog_ctx *h);

/* Destroy a context; NULL-safe.  Waits for the context's stream. */
void cog_destroy(cog_ctx *h);

/* Canonical, layout-independent state: a 64-byte header {u32 magic 'COG1',
 * u32 version 1, i32 width, height, channels, K, dtype, n_train, i64 frame},
 * then sections each padded to 64 bytes: gmm f32[P][K][C+2] (w, mu[C], var in
 * rank order), rga f32[P][C+1] (mu_r[C], var_r), table u8[P][C][16],
 * cnt u16[P][3], label u8[P] (0/1), prev f32[P][C].  For checkpoint/resume
 * and tests; synchronous; host buffers only. */
cog_status cog_canonical_bytes(const cog_params *p, size_t *bytes);
cog_status cog_export_state(cog_ctx *h, void *host_dst, size_t bytes);
cog_status cog_import_state(cog_ctx *h, const void *host_src, size_t bytes);

/* Integer prior kernel weights W[b][v] (16 x 256, row-major) for bandwidth h,
 * as used by the training kernel; host-only, needs no GPU. */
cog_status cog_kde_weights(float h, uint16_t *out);

/* Message of the last failure on h (or of the calling thread if h is NULL). */
const char *cog_last_error(const cog_ctx *h);

#ifdef __cplusplus
}
#endif
#endif /* COG_H */
