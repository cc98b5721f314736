/*
 * CPU oracle of the Cascade-of-Gaussians (CoG) background subtractor,
 * arXiv 1705.09339.  TEST INFRASTRUCTURE ONLY (see cog_oracle.h): plain,
 * slow and scalar on purpose, one pixel at a time, in the order the paper's
 * steps are stated.  Build: gcc -O2 -std=c11 -ffp-contract=off (no fast-math).
 *
 * Where the paper is silent or garbled the oracle takes the readings that the
 * design notes list (KDE form, GMM initialisation, rho, sigma^2 update, match
 * rule, sort key, confidence terms, learning-rate function).  Each function
 * below names the passage it follows.
 */
#include "cog_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NBINS 16
#define NLEVELS 256

struct orc_state {
  orc_params p;
  int64_t npix;
  int32_t n_train;  /* 0 until trained */
  int64_t frame;    /* frames consumed so far */
  float *gmm;       /* [npix][K][C+2]: w, mu[C], var -- rank order */
  float *rga;       /* [npix][C+1]: mu_r[C], var_r */
  uint8_t *table;   /* [npix][C][16] */
  uint16_t *cnt;    /* [npix][3] */
  uint8_t *label;   /* [npix] previous label */
  float *prev;      /* [npix][C] previous frame value */
  uint16_t *sat;    /* [npix] consecutive confident evaluated frames (sampling) */
  float *feat;      /* [npix][4] warm-up sums of the dominant slot: S_v, Q_v, S_w, Q_w */
  uint8_t *grp;     /* [npix] group whose shared S1 variance the pixel takes, 255: none */
  uint16_t W[NBINS][NLEVELS];
};

/* ---- scene-prior kernel weights (§2 "Scene Prior"; the KDE itself is not
 * printed in the paper: per-channel Gaussian Parzen window of bandwidth h,
 * integrated over 16 bins of 16 levels, integer weights summing to ~65535).
 * W[b][v] = rint(65535 * sum_{u=16b}^{16b+15} phi(u-v)),
 * phi(d) = exp(-d^2/(2h^2)) / sum_{e=-1024}^{1024} exp(-e^2/(2h^2)).
 * Mass that falls outside [0,255] is dropped. */
int orc_kde_weights(double h, uint16_t *out) {
  if (!(h > 0.0) || !out) return -1;
  const double den = 2.0 * h * h;
  double z = 0.0;
  for (int e = -1024; e <= 1024; ++e) z += exp(-(double)(e * e) / den);
  for (int b = 0; b < NBINS; ++b) {
    for (int v = 0; v < NLEVELS; ++v) {
      double s = 0.0;
      for (int u = NBINS * b; u < NBINS * b + NBINS; ++u) {
        int d = u - v;
        s += exp(-(double)(d * d) / den) / z;
      }
      out[b * NLEVELS + v] = (uint16_t)rint(65535.0 * s);
    }
  }
  return 0;
}

/* ---- helpers ------------------------------------------------------------- */

static float load_x(const orc_params *p, const void *frame, int64_t pix, int c) {
  if (p->dtype == ORC_U8) return (float)((const uint8_t *)frame)[pix * p->channels + c];
  return ((const float *)frame)[pix * p->channels + c];
}

/* Prior quantization q(v): u8 levels directly; f32 values mapped linearly
 * from [in_lo, in_hi) onto 256 levels (latent-space input, §3.3). */
static int quant(const orc_params *p, float v) {
  if (p->dtype == ORC_U8) return (int)v;
  float s = 256.0f / (p->in_hi - p->in_lo);
  float q = floorf((v - p->in_lo) * s);
  if (q < 0.0f) return 0;
  if (q > 255.0f) return 255;
  return (int)q;
}

/* delta = max_c |x_c - x'_c| (frame difference, §2 "Confidence Measure"). */
static float frame_delta(int C, const float *x, const float *xp) {
  float dl = 0.0f;
  for (int c = 0; c < C; ++c) {
    float d = x[c] - xp[c];
    if (d < 0.0f) d = -d;
    if (d > dl) dl = d;
  }
  return dl;
}

static float fmax0(float lo, float v) { return v < lo ? lo : v; }

/* ---- Stauffer-Grimson mixture step (§2, the update equation under "Scene
 * Prior": w <- (1-a)w + a M, mu <- (1-rho)mu + rho I, sigma^2 likewise with
 * the squared residual; diagonal -- here isotropic -- covariance). ---------- */

/* Background set: the smallest b with cumulative weight > T (else K). */
int orc_pixel_bgset(const orc_params *p, const float *comp) {
  const int F = p->channels + 2;
  float cum = 0.0f;
  for (int b = 0; b < p->K; ++b) {
    cum = cum + comp[b * F];
    if (cum > p->T) return b + 1;
  }
  return p->K;
}

/* Slot a ranks before slot b iff w_a/sigma_a > w_b/sigma_b, compared without
 * a square root as (w_a^2) sigma_b^2 > (w_b^2) sigma_a^2. */
static int ranks_before(const float *a, const float *b, int C) {
  float lhs = (a[0] * a[0]) * b[C + 1];
  float rhs = (b[0] * b[0]) * a[C + 1];
  return lhs > rhs;
}

int orc_pixel_gmmstep(const orc_params *p, float *comp, const float *x, float ae,
                      int *label, int *m_post) {
  const int K = p->K, C = p->channels, F = C + 2;
  const float lam2 = p->lambda * p->lambda;

  /* classify with the ranks and background set before the update */
  const int B = orc_pixel_bgset(p, comp);
  int m = -1;
  for (int k = 0; k < K; ++k) {
    const float *ck = comp + k * F;
    if (!(ck[0] > 0.0f)) continue;
    float d2 = 0.0f;
    for (int c = 0; c < C; ++c) {
      float d = x[c] - ck[1 + c];
      d2 = d2 + d * d;
    }
    if (d2 <= lam2 * ck[1 + C]) {
      m = k;
      break;
    }
  }
  const int lab = (m >= 0 && m < B) ? ORC_BG : ORC_FG;

  /* weights: w_k <- (1-a) w_k + a M_k */
  const float om = 1.0f - ae;
  for (int k = 0; k < K; ++k) comp[k * F] = om * comp[k * F];
  if (m >= 0) {
    float *cm = comp + m * F;
    cm[0] = cm[0] + ae;
    /* matched component: rho = a / w_m, then the mean and variance moves */
    const float rho = ae / cm[0];
    const float orho = 1.0f - rho;
    for (int c = 0; c < C; ++c) cm[1 + c] = orho * cm[1 + c] + rho * x[c];
    float s = 0.0f;
    for (int c = 0; c < C; ++c) {
      float e = x[c] - cm[1 + c];
      s = s + e * e;
    }
    cm[1 + C] = fmax0(p->var_min, orho * cm[1 + C] + rho * s);
  } else {
    /* no match: the least probable slot becomes a new component at x */
    float *cl = comp + (K - 1) * F;
    cl[0] = ae;
    for (int c = 0; c < C; ++c) cl[1 + c] = x[c];
    cl[1 + C] = p->var_init;
  }

  /* renormalise */
  float S = 0.0f;
  for (int k = 0; k < K; ++k) S = S + comp[k * F];
  for (int k = 0; k < K; ++k) comp[k * F] = comp[k * F] / S;

  /* stable insertion sort by w/sigma, following the matched slot */
  int mp = m;
  float tmp[2 + 8];
  for (int i = 1; i < K; ++i) {
    for (int j = i; j > 0 && ranks_before(comp + j * F, comp + (j - 1) * F, C); --j) {
      memcpy(tmp, comp + j * F, sizeof(float) * F);
      memcpy(comp + j * F, comp + (j - 1) * F, sizeof(float) * F);
      memcpy(comp + (j - 1) * F, tmp, sizeof(float) * F);
      if (mp == j) mp = j - 1;
      else if (mp == j - 1) mp = j;
    }
  }
  if (label) *label = lab;
  if (m_post) *m_post = mp;
  return 0;
}

/* ---- state ---------------------------------------------------------------- */

static int params_ok(const orc_params *p) {
  if (!p) return 0;
  if (p->width <= 0 || p->height <= 0) return 0;
  if (p->channels != 1 && p->channels != 3) return 0;
  if (p->K < 1 || p->K > 8) return 0;
  if (p->dtype != ORC_U8 && p->dtype != ORC_F32) return 0;
  if (p->dtype == ORC_F32 && !(p->in_hi > p->in_lo)) return 0;
  if (!(p->var_min > 0.0f) || !(p->var_init >= p->var_min)) return 0;
  if (!(p->kde_h > 0.0f)) return 0;
  if (!(p->res_e2 > 0.0f) || !(p->res_e1 <= p->res_e2)) return 0;
  if (!(p->lambda_m > 0.0f)) return 0;
  if (p->stage_mask & ORC_SAMPLE) {
    if (p->samp_window < 1 || p->samp_window > 65535) return 0;
    if (p->samp_period < 1 || p->samp_period > 65535) return 0;
    if (!(p->samp_lambda >= 0.0f)) return 0;
  }
  return 1;
}

orc_state *orc_create(const orc_params *p) {
  if (!params_ok(p)) return NULL;
  orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
  if (!s) return NULL;
  s->p = *p;
  s->npix = (int64_t)p->width * p->height;
  const int64_t P = s->npix;
  const int C = p->channels, K = p->K;
  s->gmm = (float *)calloc((size_t)(P * K * (C + 2)), sizeof(float));
  s->rga = (float *)calloc((size_t)(P * (C + 1)), sizeof(float));
  s->table = (uint8_t *)calloc((size_t)(P * C * NBINS), 1);
  s->cnt = (uint16_t *)calloc((size_t)(P * 3), sizeof(uint16_t));
  s->label = (uint8_t *)calloc((size_t)P, 1);
  s->prev = (float *)calloc((size_t)(P * C), sizeof(float));
  s->sat = (uint16_t *)calloc((size_t)P, sizeof(uint16_t));
  s->feat = (float *)calloc((size_t)P * 4, sizeof(float));
  s->grp = (uint8_t *)malloc((size_t)P);
  if (s->grp) memset(s->grp, 255, (size_t)P);
  if (!s->gmm || !s->rga || !s->table || !s->cnt || !s->label || !s->prev || !s->sat || !s->feat ||
      !s->grp ||
      orc_kde_weights((double)p->kde_h, &s->W[0][0]) != 0) {
    orc_destroy(s);
    return NULL;
  }
  return s;
}

void orc_destroy(orc_state *s) {
  if (!s) return;
  free(s->gmm);
  free(s->rga);
  free(s->table);
  free(s->cnt);
  free(s->label);
  free(s->prev);
  free(s->sat);
  free(s->feat);
  free(s->grp);
  free(s);
}

/* ---- training phase (§2 "Scene Prior", "Determining Learning Rate
 * Hyper-parameters"): per pixel over the N training frames, the integer KDE
 * bin masses, the 3-bin histogram of the frame-to-frame residue
 * (static/drift, oscillating, dynamic), and a plain mixture warm-up. ------- */
int orc_train(orc_state *s, const void *frames, int n) {
  if (!s || !frames || n < 2 || n > 65536 || s->n_train != 0) return -1;
  const orc_params *p = &s->p;
  const int C = p->channels, K = p->K, F = C + 2;
  const int64_t P = s->npix;
  const size_t fstride = (size_t)P * C * (p->dtype == ORC_U8 ? 1 : 4);
  const char *base = (const char *)frames;

  for (int64_t px = 0; px < P; ++px) {
    uint32_t acc[3][NBINS];
    uint32_t cnt[3] = {0, 0, 0};
    memset(acc, 0, sizeof(acc));
    float *comp = s->gmm + px * K * F;
    float x[3], xp[3];
    int lab = ORC_BG;
    float sv = 0.0f, qv = 0.0f, sw = 0.0f, qw = 0.0f;

    /* mixture initialisation from the first frame: one component with a
     * high initial variance, the others inactive */
    for (int c = 0; c < C; ++c) x[c] = load_x(p, base, px, c);
    for (int k = 0; k < K; ++k) {
      comp[k * F] = (k == 0) ? 1.0f : 0.0f;
      for (int c = 0; c < C; ++c) comp[k * F + 1 + c] = (k == 0) ? x[c] : 0.0f;
      comp[k * F + 1 + C] = p->var_init;
    }

    for (int j = 0; j < n; ++j) {
      const void *fr = base + (size_t)j * fstride;
      for (int c = 0; c < C; ++c) x[c] = load_x(p, fr, px, c);
      for (int c = 0; c < C; ++c) {
        int q = quant(p, x[c]);
        for (int b = 0; b < NBINS; ++b) acc[c][b] += s->W[b][q];
      }
      if (j >= 1) {
        float dl = frame_delta(C, x, xp);
        int bin = dl < p->res_e1 ? 0 : (dl < p->res_e2 ? 1 : 2);
        cnt[bin] += 1;
        orc_pixel_gmmstep(p, comp, x, p->alpha, &lab, NULL);
        /* adapted variance and weight of the dominant (rank-0) component,
         * observed after every warm-up step (grouping features) */
        const float v = comp[1 + C], w = comp[0];
        sv = sv + v;
        qv = qv + v * v;
        sw = sw + w;
        qw = qw + w * w;
      }
      for (int c = 0; c < C; ++c) xp[c] = x[c];
    }

    /* max-normalised u8 table, exact integer rounding */
    for (int c = 0; c < C; ++c) {
      uint32_t amax = 0;
      for (int b = 0; b < NBINS; ++b)
        if (acc[c][b] > amax) amax = acc[c][b];
      for (int b = 0; b < NBINS; ++b) {
        uint64_t t = amax ? ((uint64_t)255 * acc[c][b] + amax / 2) / amax : 0;
        s->table[(px * C + c) * NBINS + b] = (uint8_t)t;
      }
    }
    for (int i = 0; i < 3; ++i) s->cnt[px * 3 + i] = (uint16_t)cnt[i];

    /* running average seeded from the dominant mode; CHP state from frame N-1 */
    for (int c = 0; c < C; ++c) s->rga[px * (C + 1) + c] = comp[1 + c];
    s->rga[px * (C + 1) + C] = comp[1 + C];
    s->label[px] = (uint8_t)lab;
    for (int c = 0; c < C; ++c) s->prev[px * C + c] = xp[c];
    s->sat[px] = 0;
    s->feat[px * 4 + 0] = sv;
    s->feat[px * 4 + 1] = qv;
    s->feat[px * 4 + 2] = sw;
    s->feat[px * 4 + 3] = qw;
  }
  s->n_train = n;
  s->frame = n;
  return 0;
}

/* ---- confidence-based spatio-temporal sampling (§2 "Confidence based
 * temporal sampling", §3.2): a pixel whose value stays in its dominant mode
 * (decided by frame differencing, or by the running average within
 * samp_lambda standard deviations) for samp_window evaluated frames has a
 * saturated confidence.  Regions are blocks of ORC_BLOCK consecutive pixels:
 * when every pixel of a block is saturated, the block's cascade updates are
 * halted and it is sampled only on frames n with (n + block) divisible by
 * samp_period (the phase is staggered over blocks); on the other frames each
 * label is repeated and nothing adapts.  A pixel that is not confident on an
 * evaluated frame loses its saturation, so its block is evaluated on every
 * frame again. ------------------------------------------------------------- */
static int block_skipped(const orc_state *s, int64_t blk) {
  const orc_params *p = &s->p;
  if (!(p->stage_mask & ORC_SAMPLE)) return 0;
  if ((s->frame + blk) % p->samp_period == 0) return 0;
  const int64_t b0 = blk * ORC_BLOCK;
  const int64_t b1 = b0 + ORC_BLOCK < s->npix ? b0 + ORC_BLOCK : s->npix;
  for (int64_t px = b0; px < b1; ++px)
    if (s->sat[px] < p->samp_window) return 0;
  return 1;
}

/* ---- one frame of the rejection cascade (§2 "Cascade of Gaussians CoG",
 * "Confidence Measure"): CHP, running Gaussian average, scene-prior
 * confidence, then the full mixture; only the deciding level adapts. ------- */
int orc_step(orc_state *s, const void *frame, uint8_t *mask, int64_t *info) {
  if (!s || !frame || s->n_train == 0) return -1;
  const orc_params *p = &s->p;
  const int C = p->channels, K = p->K, F = C + 2;
  const int64_t P = s->npix;
  const float lam_r2 = p->lambda_rga * p->lambda_rga;
  const float lam_m2 = p->lambda_m * p->lambda_m;
  const float oar = 1.0f - p->alpha_rga;
  const float pden = (C == 3) ? 16581375.0f : 255.0f;  /* 255^C */
  const float nm1 = (float)(s->n_train - 1);
  const float lam_s2 = p->samp_lambda * p->samp_lambda;
  int64_t n0 = 0, n1 = 0, n2 = 0, n3 = 0, n3bg = 0, nfg = 0, nskip = 0;
  int skip = 0;

  for (int64_t px = 0; px < P; ++px) {
    if (px % ORC_BLOCK == 0) skip = block_skipped(s, px / ORC_BLOCK);
    if (skip) {
      /* halted: the label is repeated, no level runs, nothing adapts */
      const int lab = s->label[px];
      nskip++;
      if (lab == ORC_FG) nfg++;
      if (mask) mask[px] = lab == ORC_FG ? 255 : 0;
      continue;
    }
    float x[3];
    int confident = 0;
    for (int c = 0; c < C; ++c) x[c] = load_x(p, frame, px, c);
    float *xp = s->prev + px * C;
    float *rg = s->rga + px * (C + 1);
    float *comp = s->gmm + px * K * F;
    const int shared = s->grp[px] != 255; /* the S1 variance is the group's, fixed */
    int lab;

    /* S0: consistent hypothesis propagation (frame differencing) */
    const float dl = frame_delta(C, x, xp);
    if ((p->stage_mask & ORC_FD) && dl <= p->tau_fd) {
      lab = s->label[px];
      n0++;
      confident = 1;
      goto done;
    }
    /* S1: running Gaussian average */
    float dr2 = 0.0f;
    for (int c = 0; c < C; ++c) {
      float d = x[c] - rg[c];
      dr2 = dr2 + d * d;
    }
    if ((p->stage_mask & ORC_RGA) && dr2 <= lam_r2 * rg[C]) {
      lab = ORC_BG;
      confident = dr2 <= lam_s2 * rg[C];
      for (int c = 0; c < C; ++c) rg[c] = oar * rg[c] + p->alpha_rga * x[c];
      float sr = 0.0f;
      for (int c = 0; c < C; ++c) {
        float e = x[c] - rg[c];
        sr = sr + e * e;
      }
      if (!shared) rg[C] = fmax0(p->var_min, oar * rg[C] + p->alpha_rga * sr);
      n1++;
      goto done;
    }
    /* S2: scene prior lookup and confidence C = aP + bD + gM */
    float conf = 0.0f;
    if (p->stage_mask & ORC_KDE) {
      const uint8_t *tb = s->table + px * C * NBINS;
      uint32_t prod = 1;
      for (int c = 0; c < C; ++c) prod = prod * tb[c * NBINS + (quant(p, x[c]) >> 4)];
      const float ph = (float)prod / pden;
      const uint16_t *ct = s->cnt + px * 3;
      float a = (float)ct[0] / nm1;
      const float b = (float)ct[1] / nm1;
      const float g = (float)ct[2] / nm1;
      if (ph < p->p_null) a = 0.0f; /* prior nullified */
      const float dh = fmax0(0.0f, 1.0f - dl / p->res_e2);
      const float mh = fmax0(0.0f, 1.0f - dr2 / (lam_m2 * rg[C]));
      conf = (a * ph + b * dh) + g * mh;
      if (conf >= p->conf_thr) {
        lab = ORC_BG;
        n2++;
        goto done;
      }
    }
    /* S3: full mixture with the confidence-driven learning rate */
    {
      const float ae = p->alpha * (1.0f - p->kappa_alpha * conf);
      int mp = -1;
      orc_pixel_gmmstep(p, comp, x, ae, &lab, &mp);
      n3++;
      if (lab == ORC_BG) {
        n3bg++;
        for (int c = 0; c < C; ++c) rg[c] = comp[mp * F + 1 + c];
        if (!shared) rg[C] = comp[mp * F + 1 + C];
      }
    }
  done:
    if (lab == ORC_FG) nfg++;
    if (mask) mask[px] = lab == ORC_FG ? 255 : 0;
    s->label[px] = (uint8_t)lab;
    for (int c = 0; c < C; ++c) xp[c] = x[c];
    if (p->stage_mask & ORC_SAMPLE)
      s->sat[px] = confident ? (uint16_t)(s->sat[px] < 65535 ? s->sat[px] + 1 : 65535) : 0;
  }
  if (info) {
    info[0] = s->frame;
    info[1] = n0;
    info[2] = n1;
    info[3] = n2;
    info[4] = n3;
    info[5] = n3bg;
    info[6] = nfg;
    info[7] = ((double)n3 > (double)p->illum_frac * (double)P) ? 1 : 0;
    info[8] = nskip;
  }
  s->frame++;
  return 0;
}

/* ---- plain Stauffer-Grimson baseline (initialised on frame 0 by the training
 * warm-up, then one mixture step per frame with the fixed rate alpha) ------- */
int orc_gmm_step(orc_state *s, const void *frame, uint8_t *mask) {
  if (!s || !frame || s->n_train == 0) return -1;
  const orc_params *p = &s->p;
  const int C = p->channels, K = p->K, F = C + 2;
  for (int64_t px = 0; px < s->npix; ++px) {
    float x[3];
    int lab;
    for (int c = 0; c < C; ++c) x[c] = load_x(p, frame, px, c);
    orc_pixel_gmmstep(p, s->gmm + px * K * F, x, p->alpha, &lab, NULL);
    if (mask) mask[px] = lab == ORC_FG ? 255 : 0;
    s->label[px] = (uint8_t)lab;
    for (int c = 0; c < C; ++c) s->prev[px * C + c] = x[c];
  }
  s->frame++;
  return 0;
}

/* ---- spatio-temporal grouping (§2 "Clustering Similar Background"):
 * steps 1-3 give per pixel the temporal variance of the dominant mode's
 * adapted variance and weight over the training warm-up (the diagonal of
 * the paper's Cov(V), Cov(R)); step 4 is K-means with K = 3; step 5 / eq. 3
 * keeps a pixel in its cluster when its features lie within one standard
 * deviation of the cluster's mean. -------------------------------------- */
static uint32_t var_key(float S, float Q, float n) {
  const float m = S / n;
  float var = Q / n - m * m;
  if (!(var > 0.0f)) var = 0.0f;
  uint32_t u;
  memcpy(&u, &var, 4);
  return u >> 16;
}

int orc_group_keys(const orc_state *s, uint32_t *keys) {
  if (!s || !keys || s->n_train < 2) return -1;
  const float n = (float)(s->n_train - 1);
  for (int64_t px = 0; px < s->npix; ++px) {
    const float *f = s->feat + px * 4;
    keys[px * 2 + 0] = var_key(f[0], f[1], n);
    keys[px * 2 + 1] = var_key(f[2], f[3], n);
  }
  return 0;
}

static int64_t dist2(const uint32_t *k, const int64_t *c) {
  const int64_t a = (int64_t)k[0] - c[0], b = (int64_t)k[1] - c[1];
  return a * a + b * b;
}

int orc_group(const orc_state *s, uint8_t *map, double *info) {
  if (!s || s->n_train < 2) return -1;
  uint32_t *keys = (uint32_t *)malloc((size_t)s->npix * 2 * sizeof(uint32_t));
  if (!keys) return -1;
  orc_group_keys(s, keys);
  const int rc = orc_group_run(keys, s->npix, map, info);
  free(keys);
  return rc;
}

int orc_group_run(const uint32_t *keys, int64_t P, uint8_t *map, double *info) {
  if (!keys || P < 1) return -1;
  const int G = ORC_NGROUPS;
  uint8_t *asg = (uint8_t *)malloc((size_t)P);
  if (!asg) return -1;
  /* initial centres: the minimum, the floor of the mean and the maximum of
   * each key */
  int64_t c[ORC_NGROUPS][2];
  for (int d = 0; d < 2; ++d) {
    uint32_t lo = keys[d], hi = keys[d];
    uint64_t sum = 0;
    for (int64_t px = 0; px < P; ++px) {
      const uint32_t v = keys[px * 2 + d];
      lo = v < lo ? v : lo;
      hi = v > hi ? v : hi;
      sum += v;
    }
    c[0][d] = lo;
    c[1][d] = (int64_t)(sum / (uint64_t)P);
    c[2][d] = hi;
  }
  /* Lloyd iterations: nearest centre (lowest index on ties), centres move
   * to the floor of their members' mean; stop when no assignment changes */
  int it = 0;
  for (int64_t px = 0; px < P; ++px) asg[px] = 255;
  for (it = 1; it <= ORC_GROUP_ITERS; ++it) {
    int64_t changed = 0;
    uint64_t cnt[ORC_NGROUPS] = {0}, sum[ORC_NGROUPS][2] = {{0}};
    for (int64_t px = 0; px < P; ++px) {
      int best = 0;
      int64_t bd = dist2(keys + px * 2, c[0]);
      for (int g = 1; g < G; ++g) {
        const int64_t d = dist2(keys + px * 2, c[g]);
        if (d < bd) {
          bd = d;
          best = g;
        }
      }
      if (asg[px] != best) changed++;
      asg[px] = (uint8_t)best;
      cnt[best]++;
      sum[best][0] += keys[px * 2];
      sum[best][1] += keys[px * 2 + 1];
    }
    if (changed == 0) break;
    for (int g = 0; g < G; ++g)
      if (cnt[g])
        for (int d = 0; d < 2; ++d) c[g][d] = (int64_t)(sum[g][d] / cnt[g]);
  }
  if (it > ORC_GROUP_ITERS) it = ORC_GROUP_ITERS;
  /* eq. 3: one standard deviation around each cluster's member mean */
  double mean[ORC_NGROUPS][2], sd[ORC_NGROUPS][2];
  uint64_t cnt[ORC_NGROUPS] = {0};
  uint64_t s1[ORC_NGROUPS][2] = {{0}}, s2[ORC_NGROUPS][2] = {{0}};
  for (int64_t px = 0; px < P; ++px) {
    const int g = asg[px];
    cnt[g]++;
    for (int d = 0; d < 2; ++d) {
      const uint64_t v = keys[px * 2 + d];
      s1[g][d] += v;
      s2[g][d] += v * v;
    }
  }
  for (int g = 0; g < G; ++g)
    for (int d = 0; d < 2; ++d) {
      if (!cnt[g]) {
        mean[g][d] = sd[g][d] = 0.0;
        continue;
      }
      const double n = (double)cnt[g];
      mean[g][d] = (double)s1[g][d] / n;
      double var = (double)s2[g][d] / n - mean[g][d] * mean[g][d];
      sd[g][d] = var > 0.0 ? sqrt(var) : 0.0;
    }
  uint64_t grouped[ORC_NGROUPS] = {0};
  for (int64_t px = 0; px < P; ++px) {
    const int g = asg[px];
    int in = 1;
    for (int d = 0; d < 2; ++d) {
      const double e = (double)keys[px * 2 + d] - mean[g][d];
      if (!(fabs(e) <= sd[g][d])) in = 0;
    }
    if (in) grouped[g]++;
    if (map) map[px] = in ? (uint8_t)g : 255;
  }
  if (info) {
    info[0] = it;
    for (int g = 0; g < G; ++g) {
      double *o = info + 1 + 8 * g;
      o[0] = (double)cnt[g];
      o[1] = (double)c[g][0];
      o[2] = (double)c[g][1];
      o[3] = mean[g][0];
      o[4] = sd[g][0];
      o[5] = mean[g][1];
      o[6] = sd[g][1];
      o[7] = (double)grouped[g];
    }
  }
  free(asg);
  return 0;
}

/* ---- one shared parameter set per group (§2 "Clustering Similar
 * Background", the list's last item and eq. 3): the pixels of a group share
 * the variance of the first, dominant cascade level (the running Gaussian
 * average), fitted once as the mean of the members' variances, so that
 * the region has one variance parameter and its pixels no longer update it.
 * The mean is taken exactly on a fixed-point grid: each member's variance
 * rounded to a multiple of 2^-16 (binary64 rint, ties to even), summed as
 * integers, then divided once in binary64 and rounded to binary32, and held
 * at var_min or above.  Means keep adapting per pixel.  map: group 0..2 per
 * pixel (255: not grouped), e.g. the map of orc_group; NULL ungroups every
 * pixel, which then adapts its variance again from the value it holds.
 * gvar (may be NULL): the 3 shared variances (0 for an empty group). ------ */
int orc_group_share(orc_state *s, const uint8_t *map, float *gvar) {
  if (!s || s->n_train == 0) return -1;
  const int C = s->p.channels;
  const int64_t P = s->npix;
  uint64_t cnt[ORC_NGROUPS] = {0}, sum[ORC_NGROUPS] = {0};
  float v[ORC_NGROUPS] = {0.0f, 0.0f, 0.0f};
  if (map) {
    for (int64_t px = 0; px < P; ++px) {
      const int g = map[px];
      if (g == 255) continue;
      if (g >= ORC_NGROUPS) return -1;
      const double q = rint((double)s->rga[px * (C + 1) + C] * 65536.0);
      if (!(q >= 0.0 && q < 9007199254740992.0)) return -1; /* 2^53 */
      cnt[g]++;
      sum[g] += (uint64_t)q;
    }
    for (int g = 0; g < ORC_NGROUPS; ++g) {
      if (!cnt[g]) continue;
      const float m = (float)((double)sum[g] / 65536.0 / (double)cnt[g]);
      v[g] = fmax0(s->p.var_min, m);
    }
  }
  orc_group_set(s, map, v);
  if (gvar)
    for (int g = 0; g < ORC_NGROUPS; ++g) gvar[g] = v[g];
  return 0;
}

/* The members of each group take the given shared variance gvar[g] (no
 * fitting); the others keep their own.  map NULL ungroups every pixel. */
int orc_group_set(orc_state *s, const uint8_t *map, const float *gvar) {
  if (!s || s->n_train == 0 || (map && !gvar)) return -1;
  const int C = s->p.channels;
  const int64_t P = s->npix;
  if (map)
    for (int64_t px = 0; px < P; ++px)
      if (map[px] != 255 && map[px] >= ORC_NGROUPS) return -1;
  for (int64_t px = 0; px < P; ++px) {
    const int g = map ? map[px] : 255;
    s->grp[px] = (uint8_t)g;
    if (g != 255) s->rga[px * (C + 1) + C] = gvar[g];
  }
  return 0;
}

/* ---- canonical export: 64-byte header (version 3), then sections each
 * padded to 64 B: gmm f32[P][K][C+2], rga f32[P][C+1], table u8[P][C][16],
 * cnt u16[P][3], label u8[P], prev f32[P][C], sat u16[P], gkey u32[P][2]
 * (the grouping keys of the training warm-up), shared u8[P] (1 where the
 * pixel takes its group's shared variance). -------------------------------- */
static size_t pad64(size_t n) { return (n + 63) & ~(size_t)63; }

size_t orc_canonical_bytes(const orc_params *p) {
  if (!params_ok(p)) return 0;
  const size_t P = (size_t)p->width * p->height;
  const size_t C = (size_t)p->channels, K = (size_t)p->K;
  return 64 + pad64(P * K * (C + 2) * 4) + pad64(P * (C + 1) * 4) + pad64(P * C * NBINS) +
         pad64(P * 3 * 2) + pad64(P) + pad64(P * C * 4) + pad64(P * 2) + pad64(P * 8) + pad64(P);
}

int orc_export(const orc_state *s, void *dst, size_t bytes) {
  if (!s || !dst) return -1;
  const orc_params *p = &s->p;
  if (bytes < orc_canonical_bytes(p)) return -1;
  const size_t P = (size_t)s->npix;
  const size_t C = (size_t)p->channels, K = (size_t)p->K;
  char *o = (char *)dst;
  memset(o, 0, orc_canonical_bytes(p));
  uint32_t hdr32[2] = {0x31474F43u, 3u};
  int32_t hdri[6] = {p->width, p->height, p->channels, p->K, p->dtype, s->n_train};
  int64_t fr = s->frame;
  memcpy(o, hdr32, 8);
  memcpy(o + 8, hdri, 24);
  memcpy(o + 32, &fr, 8);
  size_t off = 64;
  memcpy(o + off, s->gmm, P * K * (C + 2) * 4);
  off += pad64(P * K * (C + 2) * 4);
  memcpy(o + off, s->rga, P * (C + 1) * 4);
  off += pad64(P * (C + 1) * 4);
  memcpy(o + off, s->table, P * C * NBINS);
  off += pad64(P * C * NBINS);
  memcpy(o + off, s->cnt, P * 3 * 2);
  off += pad64(P * 3 * 2);
  memcpy(o + off, s->label, P);
  off += pad64(P);
  memcpy(o + off, s->prev, P * C * 4);
  off += pad64(P * C * 4);
  memcpy(o + off, s->sat, P * 2);
  off += pad64(P * 2);
  if (s->n_train >= 2) orc_group_keys(s, (uint32_t *)(o + off));
  off += pad64(P * 8);
  for (size_t px = 0; px < P; ++px) o[off + px] = s->grp[px] != 255 ? 1 : 0;
  return 0;
}
