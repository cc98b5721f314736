/*
 * CPU oracle of the Cascade-of-Gaussians (CoG) background subtractor
 * (Kiran, Das, Yogamani, "Rejection-Cascade of Gaussians", arXiv 1705.09339).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, scalar reference that
 * the HIP library is checked against.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant generator with the HIP library.
 *
 * Precision: binary32 state and arithmetic, every operation a single IEEE-754
 * round-to-nearest-even op evaluated left to right as written, no FMA
 * contraction (-ffp-contract=off), IEEE denormals, correctly rounded
 * division.  The method's discrete decisions (component match, background
 * set, sort order, cascade gates) are taken in the same precision as the
 * kernels, so the recurrence itself is carried in binary32.
 */
#ifndef COG_ORACLE_H
#define COG_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_U8 = 0, ORC_F32 = 1 };
enum { ORC_FD = 1u, ORC_RGA = 2u, ORC_KDE = 4u, ORC_SAMPLE = 8u };
enum { ORC_BG = 0, ORC_FG = 1 };

typedef struct {
  int32_t width, height, channels, K;
  int32_t dtype;            /* ORC_U8 or ORC_F32 */
  float in_lo, in_hi;       /* prior quantization range of f32 input */
  float alpha, T, lambda, var_init, var_min;
  uint32_t stage_mask;      /* ORC_FD | ORC_RGA | ORC_KDE */
  float tau_fd, lambda_rga, alpha_rga;
  float kde_h, res_e1, res_e2;
  float lambda_m, conf_thr, p_null, kappa_alpha;
  float illum_frac;
  /* confidence-based spatio-temporal sampling (stage bit ORC_SAMPLE) */
  int32_t samp_window;      /* confident frames before a pixel saturates */
  int32_t samp_period;      /* a saturated block is evaluated every samp_period frames */
  float samp_lambda;        /* confidence gate of S1 decisions, in standard deviations */
} orc_params;

typedef struct orc_state orc_state;

/* info[9] = {frame, n0, n1, n2, n3, n3_bg, n_fg, illum_flag, n_skip} */
enum { ORC_INFO_LEN = 9 };
enum { ORC_BLOCK = 64 };  /* pixels per sampling block (consecutive, row-major) */

/* Integer kernel-weight table W[b][v] (16 bins x 256 levels), row-major. */
int orc_kde_weights(double h, uint16_t *out);

orc_state *orc_create(const orc_params *p);
void orc_destroy(orc_state *s);

/* Training phase over frames[0..n-1] (frames: n x P x C, u8 or f32). */
int orc_train(orc_state *s, const void *frames, int n);
/* One cascade step; mask (P bytes, 0/255) and info may be NULL. */
int orc_step(orc_state *s, const void *frame, uint8_t *mask, int64_t *info);
/* One plain Stauffer-Grimson step on the same GMM state (no cascade). */
int orc_gmm_step(orc_state *s, const void *frame, uint8_t *mask);

/* Single-pixel GMM step on a K x (C+2) record {w, mu[C], var}, in place. */
int orc_pixel_gmmstep(const orc_params *p, float *comp, const float *x, float alpha_e,
                      int *label, int *m_post);
/* Background-set size B of a sorted record. */
int orc_pixel_bgset(const orc_params *p, const float *comp);

/* Spatio-temporal grouping of the background (§2 "Clustering Similar
 * Background - Spatio-Temporal Grouping"), after training.  Per pixel, the
 * training warm-up gives the temporal variance of the dominant component's
 * adapted variance and of its weight; each becomes an integer key (its
 * binary32 pattern >> 16, a piecewise-linear log2 scale).  Integer k-means
 * with ORC_NGROUPS clusters groups the keys; a pixel keeps its cluster if
 * both keys lie within one standard deviation of the cluster's member mean
 * (closed interval), else it is ungrouped (255).
 *   keys: P x 2 u32 (may be NULL); map: P bytes (may be NULL);
 *   info (may be NULL): ORC_GROUP_INFO doubles =
 *     {iterations, then per cluster g: count, center1, center2, mean1, sd1,
 *      mean2, sd2, grouped} */
enum { ORC_NGROUPS = 3, ORC_GROUP_ITERS = 32, ORC_GROUP_INFO = 1 + 8 * 3 };
int orc_group_keys(const orc_state *s, uint32_t *keys);
int orc_group(const orc_state *s, uint8_t *map, double *info);
/* The clustering and eq. 3 band alone, on given keys (P x 2 u32, P >= 1). */
int orc_group_run(const uint32_t *keys, int64_t P, uint8_t *map, double *info);

/* One shared parameter set per group (eq. 3 and the list before it): the
 * pixels of each group take one shared variance of the running Gaussian
 * average (S1), the exact mean of the members' variances on a 2^-16 grid,
 * at least var_min, and stop adapting it; means still adapt per pixel.
 * map: P bytes, group 0..2 or 255 (not grouped); NULL ungroups all.
 * gvar (may be NULL): the 3 shared variances, 0 for an empty group. */
int orc_group_share(orc_state *s, const uint8_t *map, float *gvar);
/* The sharing alone with given values: members of group g take gvar[g]. */
int orc_group_set(orc_state *s, const uint8_t *map, const float *gvar);

size_t orc_canonical_bytes(const orc_params *p);
int orc_export(const orc_state *s, void *dst, size_t bytes);

#ifdef __cplusplus
}
#endif
#endif
