// gfx950 kernels of the Cascade-of-Gaussians background subtractor
// (arXiv 1705.09339): prior training, the fused rejection cascade and the
// plain mixture baseline.
//
// Numerics: every floating-point expression below is evaluated as written,
// one binary32 round-to-nearest-even operation at a time (the library is
// built with -ffp-contract=off, IEEE denormals and correctly rounded
// division), so the discrete decisions of the method -- component match,
// background set, rank order, cascade gates -- are reproducible bit for bit.
// There are no transcendental functions on the per-frame path; the rank key
// w/sigma is compared as w_a^2 sigma_b^2 > w_b^2 sigma_a^2.
#include "cog_device.h"

namespace cog {
namespace {

// ----------------------------------------------------------------------------
// Per-pixel Stauffer-Grimson mixture held in registers.
template <int C, int K>
struct Mix {
  float w[K];
  float var[K];
  float mu[K][C];
};

template <int C, int K>
__device__ __forceinline__ void mix_init(Mix<C, K> &s, const float (&x)[C], float var_init) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s.w[k] = (k == 0) ? 1.0f : 0.0f;
    s.var[k] = var_init;
#pragma unroll
    for (int c = 0; c < C; ++c) s.mu[k][c] = (k == 0) ? x[c] : 0.0f;
  }
}

// Background set B: the smallest b whose cumulative weight exceeds T.
template <int C, int K>
__device__ __forceinline__ int mix_bgset(const Mix<C, K> &s, float T) {
  float cum = 0.0f;
  int B = K;
  bool closed = false;
#pragma unroll
  for (int b = 0; b < K; ++b) {
    cum = cum + s.w[b];
    if (!closed && cum > T) {
      B = b + 1;
      closed = true;
    }
  }
  return B;
}

// One mixture step (§2, the update equation under "Scene Prior"):
// classify against the pre-update ranks, w <- (1-a)w + aM, the matched
// component's mean and variance move with rho = a / w_m, an unmatched value
// replaces the last-ranked slot, weights are renormalised and the slots are
// re-ranked by w/sigma (stable).  Returns the label (1 = foreground) and the
// matched slot's rank after the re-sort (-1 when nothing matched).
template <int C, int K>
__device__ __forceinline__ void mix_step(Mix<C, K> &s, const float (&x)[C], float ae,
                                         const KParams &kp, int &label, int &mpost) {
  const int B = mix_bgset<C, K>(s, kp.T);
  int m = -1;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float d2 = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float d = x[c] - s.mu[k][c];
      d2 = d2 + d * d;
    }
    const bool hit = (s.w[k] > 0.0f) && (d2 <= kp.lam2 * s.var[k]);
    if (m < 0 && hit) m = k;
  }
  label = (m >= 0 && m < B) ? 0 : 1;

  const float om = 1.0f - ae;
#pragma unroll
  for (int k = 0; k < K; ++k) s.w[k] = om * s.w[k];
  if (m >= 0) {
    float wm = s.w[0], vm = s.var[0], mm[C];
#pragma unroll
    for (int c = 0; c < C; ++c) mm[c] = s.mu[0][c];
#pragma unroll
    for (int k = 1; k < K; ++k) {
      if (m == k) {
        wm = s.w[k];
        vm = s.var[k];
#pragma unroll
        for (int c = 0; c < C; ++c) mm[c] = s.mu[k][c];
      }
    }
    wm = wm + ae;
    const float rho = ae / wm;
    const float orho = 1.0f - rho;
#pragma unroll
    for (int c = 0; c < C; ++c) mm[c] = orho * mm[c] + rho * x[c];
    float sse = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float e = x[c] - mm[c];
      sse = sse + e * e;
    }
    const float v = orho * vm + rho * sse;
    vm = v < kp.var_min ? kp.var_min : v;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (m == k) {
        s.w[k] = wm;
        s.var[k] = vm;
#pragma unroll
        for (int c = 0; c < C; ++c) s.mu[k][c] = mm[c];
      }
    }
  } else {
    s.w[K - 1] = ae;
    s.var[K - 1] = kp.var_init;
#pragma unroll
    for (int c = 0; c < C; ++c) s.mu[K - 1][c] = x[c];
  }

  float S = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) S = S + s.w[k];
#pragma unroll
  for (int k = 0; k < K; ++k) s.w[k] = s.w[k] / S;

  // Insertion sort written as a fixed compare-exchange sequence: inside the
  // already ranked prefix no pair ranks out of order (the key comparison is
  // antisymmetric), so the extra comparisons never exchange and the result
  // equals the early-exit insertion sort.
  int mp = m;
#pragma unroll
  for (int i = 1; i < K; ++i) {
#pragma unroll
    for (int j = i; j > 0; --j) {
      const float lhs = (s.w[j] * s.w[j]) * s.var[j - 1];
      const float rhs = (s.w[j - 1] * s.w[j - 1]) * s.var[j];
      if (lhs > rhs) {
        float t = s.w[j];
        s.w[j] = s.w[j - 1];
        s.w[j - 1] = t;
        t = s.var[j];
        s.var[j] = s.var[j - 1];
        s.var[j - 1] = t;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          t = s.mu[j][c];
          s.mu[j][c] = s.mu[j - 1][c];
          s.mu[j - 1][c] = t;
        }
        mp = (mp == j) ? j - 1 : ((mp == j - 1) ? j : mp);
      }
    }
  }
  mpost = mp;
}

// ---- mixture record layouts ------------------------------------------------
// Cascade: one record of rec_floats(C,K) floats per pixel, {w[K], var[K],
// mu[K][C]}, 16-byte aligned, so a lone survivor reads one or two lines.
template <int C, int K>
__device__ __forceinline__ void rec_load(const float *rec, Mix<C, K> &s) {
  constexpr int R = rec_floats(C, K);
  float r[R];
  const float4 *r4 = reinterpret_cast<const float4 *>(rec);
#pragma unroll
  for (int i = 0; i < R / 4; ++i) {
    const float4 v = r4[i];
    r[4 * i] = v.x;
    r[4 * i + 1] = v.y;
    r[4 * i + 2] = v.z;
    r[4 * i + 3] = v.w;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s.w[k] = r[k];
    s.var[k] = r[K + k];
#pragma unroll
    for (int c = 0; c < C; ++c) s.mu[k][c] = r[2 * K + k * C + c];
  }
}

template <int C, int K>
__device__ __forceinline__ void rec_store(float *rec, const Mix<C, K> &s) {
  constexpr int R = rec_floats(C, K);
  float r[R];
#pragma unroll
  for (int i = 0; i < R; ++i) r[i] = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    r[k] = s.w[k];
    r[K + k] = s.var[k];
#pragma unroll
    for (int c = 0; c < C; ++c) r[2 * K + k * C + c] = s.mu[k][c];
  }
  float4 *r4 = reinterpret_cast<float4 *>(rec);
#pragma unroll
  for (int i = 0; i < R / 4; ++i) r4[i] = make_float4(r[4 * i], r[4 * i + 1], r[4 * i + 2], r[4 * i + 3]);
}

// Baseline: the same fields in groups of 64 pixels (field-major inside a
// group), so that a wave reading one field touches one 256-byte segment.
template <int C, int K>
__device__ __forceinline__ float *grp_field(float *g, int64_t p, int f) {
  constexpr int R = rec_floats(C, K);
  return g + (((p >> 6) * R + f) << 6) + (p & 63);
}

template <int C, int K>
__device__ __forceinline__ void grp_load(float *g, int64_t p, Mix<C, K> &s) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s.w[k] = *grp_field<C, K>(g, p, k);
    s.var[k] = *grp_field<C, K>(g, p, K + k);
#pragma unroll
    for (int c = 0; c < C; ++c) s.mu[k][c] = *grp_field<C, K>(g, p, 2 * K + k * C + c);
  }
}

template <int C, int K>
__device__ __forceinline__ void grp_store(float *g, int64_t p, const Mix<C, K> &s) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    *grp_field<C, K>(g, p, k) = s.w[k];
    *grp_field<C, K>(g, p, K + k) = s.var[k];
#pragma unroll
    for (int c = 0; c < C; ++c) *grp_field<C, K>(g, p, 2 * K + k * C + c) = s.mu[k][c];
  }
}

// ---- input -----------------------------------------------------------------
template <int C, bool F32>
__device__ __forceinline__ void load_px(const void *base, int64_t p, float (&x)[C]) {
  if constexpr (F32) {
    const float *q = static_cast<const float *>(base) + p * C;
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = q[c];
  } else {
    const uint8_t *q = static_cast<const uint8_t *>(base) + p * C;
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = (float)q[c];
  }
}

template <int C, bool F32>
__device__ __forceinline__ void store_px(void *base, int64_t p, const float (&x)[C]) {
  if constexpr (F32) {
    float *q = static_cast<float *>(base) + p * C;
#pragma unroll
    for (int c = 0; c < C; ++c) q[c] = x[c];
  } else {
    uint8_t *q = static_cast<uint8_t *>(base) + p * C;
#pragma unroll
    for (int c = 0; c < C; ++c) q[c] = (uint8_t)x[c];
  }
}

template <int C, bool F32>
__device__ __forceinline__ const void *frame_ptr(const void *x, int64_t stride, int f) {
  if constexpr (F32) return static_cast<const float *>(x) + (int64_t)f * stride;
  return static_cast<const uint8_t *>(x) + (int64_t)f * stride;
}

// Prior quantisation: u8 levels directly; f32 values onto 256 levels.
template <bool F32>
__device__ __forceinline__ int quant(float v, const KParams &kp) {
  if constexpr (!F32) {
    return (int)v;
  } else {
    const float q = floorf((v - kp.in_lo) * kp.q_scale);
    if (q < 0.0f) return 0;
    if (q > 255.0f) return 255;
    return (int)q;
  }
}

template <int C>
__device__ __forceinline__ float frame_delta(const float (&x)[C], const float (&xp)[C]) {
  float dl = 0.0f;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    float d = x[c] - xp[c];
    d = d < 0.0f ? -d : d;
    dl = d > dl ? d : dl;
  }
  return dl;
}

__device__ __forceinline__ int lane_prefix(unsigned long long bal) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
}

// ============================================================================
// Training phase: one thread per pixel walks the N training frames.
//  - integer KDE bin masses acc[c][b] += W[b][q(x)] (weights staged in LDS,
//    level-major so one level's 16 weights are two 16-byte reads),
//  - the residue histogram over max_c |x_j - x_{j-1}|,
//  - the mixture warm-up (initialised from frame 0, stepped on 1..N-1).
// Then the max-normalised u8 table, counts, mixture, running average (from
// the dominant mode), previous frame and label are written once.
template <int C, int K, bool F32>
__global__ __launch_bounds__(kNT) void k_train(Buffers b, const void *frames, int64_t stride,
                                               int n, KParams kp, int with_prior, int aos) {
  __shared__ uint4 s_w[256 * kBins * 2 / 16];
  for (int i = threadIdx.x; i < 256 * kBins * 2 / 16; i += kNT)
    s_w[i] = reinterpret_cast<const uint4 *>(b.kdew)[i];
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const bool valid = p < b.P;
  bool lab = false;
  if (valid) {
    uint32_t acc[C][kBins];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q = 0; q < kBins; ++q) acc[c][q] = 0u;
    uint32_t cnt0 = 0, cnt1 = 0, cnt2 = 0;
    float x[C], xp[C];
    Mix<C, K> m;
    load_px<C, F32>(frames, p, x);
    mix_init<C, K>(m, x, kp.var_init);
    for (int j = 0; j < n; ++j) {
      load_px<C, F32>(frame_ptr<C, F32>(frames, stride, j), p, x);
      if (with_prior) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const int v = quant<F32>(x[c], kp);
          const uint4 lo = s_w[2 * v], hi = s_w[2 * v + 1];
          const uint32_t wd[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            acc[c][2 * q] += wd[q] & 0xffffu;
            acc[c][2 * q + 1] += wd[q] >> 16;
          }
        }
      }
      if (j >= 1) {
        if (with_prior) {
          const float dl = frame_delta<C>(x, xp);
          if (dl < kp.res_e1) cnt0++;
          else if (dl < kp.res_e2) cnt1++;
          else cnt2++;
        }
        int l, mp;
        mix_step<C, K>(m, x, kp.alpha, kp, l, mp);
        lab = l != 0;
      }
#pragma unroll
      for (int c = 0; c < C; ++c) xp[c] = x[c];
    }

    if (with_prior) {
      constexpr int PB = prior_bytes(C);
      uint32_t words[PB / 4];
#pragma unroll
      for (int i = 0; i < PB / 4; ++i) words[i] = 0u;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        uint32_t amax = 0;
#pragma unroll
        for (int q = 0; q < kBins; ++q) amax = acc[c][q] > amax ? acc[c][q] : amax;
#pragma unroll
        for (int q = 0; q < kBins; ++q) {
          const uint32_t t =
              amax ? (uint32_t)((255ull * acc[c][q] + (amax >> 1)) / amax) : 0u;
          const int byte = c * kBins + q;
          words[byte >> 2] |= (t & 0xffu) << (8 * (byte & 3));
        }
      }
      words[(C * kBins) / 4] = (cnt0 & 0xffffu) | (cnt1 << 16);
      words[(C * kBins) / 4 + 1] = cnt2 & 0xffffu;
      uint4 *dst = reinterpret_cast<uint4 *>(b.prior + p * PB);
#pragma unroll
      for (int i = 0; i < PB / 16; ++i)
        dst[i] = make_uint4(words[4 * i], words[4 * i + 1], words[4 * i + 2], words[4 * i + 3]);

      constexpr int RG = rga_floats(C);
      float *rg = b.rga + p * RG;
#pragma unroll
      for (int c = 0; c < C; ++c) rg[c] = m.mu[0][c];
      rg[C] = m.var[0];
    }
    if (aos) rec_store<C, K>(b.gmm + p * rec_floats(C, K), m);
    else grp_store<C, K>(b.gmm, p, m);
    store_px<C, F32>(b.prev, p, xp);
  }
  const unsigned long long bal = __ballot(lab);
  const int64_t w0 = p - lane;
  if (lane == 0 && w0 < b.P) b.labels[w0 >> 6] = bal;
}

// ============================================================================
// The fused rejection cascade (§2 "Cascade of Gaussians CoG", "Confidence
// Measure"), one workgroup per tile of kNT*PPT pixels, for nframes
// consecutive frames.  Per frame:
//   dense  : S0 frame difference and S1 running average for every pixel, in
//            the owning thread's registers;
//   list A : survivors of S1 compacted into LDS (wave ballot, lane prefix by
//            mbcnt, prefix over waves) in pixel order;
//   S2     : scene-prior lookup and confidence over list A; survivors
//            compacted again into list B;
//   S3     : the full mixture over list B (records read and written in HBM);
//   finish : the owners take the labels and running-average re-seeds back,
//            write the mask and count the level occupancy.
// The dense state (previous value, label, running average) stays in
// registers across the frames of one launch; only the deciding level adapts.
template <int C, int K, bool F32, int PPT>
__global__ __launch_bounds__(kNT) void k_cascade(Buffers b, Frames fr, KParams kp) {
  constexpr int TILE = kNT * PPT;
  constexpr int R = rec_floats(C, K);
  constexpr int RG = rga_floats(C);
  constexpr int PB = prior_bytes(C);
  __shared__ float s_x[TILE * C];
  __shared__ float s_dl[TILE];
  __shared__ float s_dr2[TILE];
  __shared__ float s_var[TILE];
  __shared__ float s_conf[TILE];
  __shared__ float s_rg[TILE * (C + 1)];
  __shared__ uint16_t s_la[TILE];
  __shared__ uint16_t s_lb[TILE];
  __shared__ uint8_t s_res[TILE];  // bit0 foreground, bit1 re-seed, bits 2-3 stage
  __shared__ int s_cnt[kNW * PPT];
  __shared__ int s_cnt2[kNW];
  __shared__ uint32_t s_stat[2][kStat];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t tile0 = (int64_t)blockIdx.x * TILE;
  const bool fd_on = (kp.stage_mask & 1u) != 0;
  const bool rga_on = (kp.stage_mask & 2u) != 0;
  const bool kde_on = (kp.stage_mask & 4u) != 0;

  float xp[PPT][C], rmu[PPT][C], rvar[PPT];
  bool lab[PPT], dirty[PPT], valid[PPT];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int64_t p = tile0 + j * kNT + tid;
    valid[j] = p < b.P;
    dirty[j] = false;
    lab[j] = false;
    rvar[j] = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) xp[j][c] = rmu[j][c] = 0.0f;
    if (valid[j]) {
      const unsigned long long word = b.labels[p >> 6];
      lab[j] = ((word >> lane) & 1ull) != 0;
      load_px<C, F32>(b.prev, p, xp[j]);
      const float *rg = b.rga + p * RG;
#pragma unroll
      for (int c = 0; c < C; ++c) rmu[j][c] = rg[c];
      rvar[j] = rg[C];
    }
  }
  if (tid < 2 * kStat) (&s_stat[0][0])[tid] = 0u;

  for (int f = 0; f < fr.nframes; ++f) {
    const void *xf = frame_ptr<C, F32>(fr.x, fr.stride, f);
    float x[PPT][C];
    int st[PPT], pre[PPT];
    bool surv[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int64_t p = tile0 + j * kNT + tid;
      const int li = j * kNT + tid;
      st[j] = -1;
      surv[j] = false;
#pragma unroll
      for (int c = 0; c < C; ++c) x[j][c] = 0.0f;
      if (valid[j]) {
        load_px<C, F32>(xf, p, x[j]);
        const float dl = frame_delta<C>(x[j], xp[j]);
        if (fd_on && dl <= kp.tau_fd) {
          st[j] = 0;  // S0: repeat the previous label
        } else {
          float dr2 = 0.0f;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const float d = x[j][c] - rmu[j][c];
            dr2 = dr2 + d * d;
          }
          if (rga_on && dr2 <= kp.lam_r2 * rvar[j]) {
            st[j] = 1;  // S1: background, the running average adapts
            lab[j] = false;
#pragma unroll
            for (int c = 0; c < C; ++c)
              rmu[j][c] = kp.one_m_alpha_rga * rmu[j][c] + kp.alpha_rga * x[j][c];
            float sr = 0.0f;
#pragma unroll
            for (int c = 0; c < C; ++c) {
              const float e = x[j][c] - rmu[j][c];
              sr = sr + e * e;
            }
            const float v = kp.one_m_alpha_rga * rvar[j] + kp.alpha_rga * sr;
            rvar[j] = v < kp.var_min ? kp.var_min : v;
            dirty[j] = true;
          } else {
            surv[j] = true;
#pragma unroll
            for (int c = 0; c < C; ++c) s_x[li * C + c] = x[j][c];
            s_dl[li] = dl;
            s_dr2[li] = dr2;
            s_var[li] = rvar[j];
          }
        }
      }
      const unsigned long long bal = __ballot(surv[j]);
      if (lane == 0) s_cnt[j * kNW + wave] = (int)__popcll(bal);
      pre[j] = lane_prefix(bal);
    }
    __syncthreads();
    if (tid == 0) {
      if (f > 0) {
        uint32_t *sp = &s_stat[(f - 1) & 1][0];
        if (fr.partials) {
          uint32_t *dst = fr.partials + ((int64_t)(f - 1) * fr.nslots + blockIdx.x) * kStat;
#pragma unroll
          for (int k = 0; k < kStat; ++k) dst[k] = sp[k];
        }
#pragma unroll
        for (int k = 0; k < kStat; ++k) sp[k] = 0u;
      }
    }
    int nA = 0, off[PPT];
#pragma unroll
    for (int q = 0; q < kNW * PPT; ++q) {
      const int cq = s_cnt[q];
#pragma unroll
      for (int j = 0; j < PPT; ++j)
        if (q == j * kNW + wave) off[j] = nA;
      nA += cq;
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j)
      if (surv[j]) s_la[off[j] + pre[j]] = (uint16_t)(j * kNT + tid);
    __syncthreads();

    // S2: scene prior and confidence; compaction of the survivors into list B.
    int nB = 0;
    for (int r0 = 0; r0 < nA; r0 += kNT) {
      const int i = r0 + tid;
      bool go3 = false;
      int li = 0;
      if (i < nA) {
        li = s_la[i];
        float conf = 0.0f;
        bool accept = false;
        if (kde_on) {
          const uint8_t *rec = b.prior + (tile0 + li) * PB;
          uint32_t prod = 1u;
#pragma unroll
          for (int c = 0; c < C; ++c)
            prod = prod * (uint32_t)rec[c * kBins + (quant<F32>(s_x[li * C + c], kp) >> 4)];
          const float ph = (float)prod / (C == 3 ? 16581375.0f : 255.0f);
          const uint16_t *cn = reinterpret_cast<const uint16_t *>(rec + C * kBins);
          float a = (float)cn[0] / kp.nm1;
          const float bw = (float)cn[1] / kp.nm1;
          const float g = (float)cn[2] / kp.nm1;
          if (ph < kp.p_null) a = 0.0f;  // prior nullified
          float dh = 1.0f - s_dl[li] / kp.res_e2;
          dh = dh < 0.0f ? 0.0f : dh;
          float mh = 1.0f - s_dr2[li] / (kp.lam_m2 * s_var[li]);
          mh = mh < 0.0f ? 0.0f : mh;
          conf = (a * ph + bw * dh) + g * mh;
          accept = conf >= kp.conf_thr;
        }
        if (accept) {
          s_res[li] = (uint8_t)(2 << 2);
        } else {
          go3 = true;
          s_conf[li] = conf;
        }
      }
      const unsigned long long bal = __ballot(go3);
      if (lane == 0) s_cnt2[wave] = (int)__popcll(bal);
      __syncthreads();
      int base = 0, tot = 0;
#pragma unroll
      for (int w = 0; w < kNW; ++w) {
        if (w == wave) base = tot;
        tot += s_cnt2[w];
      }
      if (go3) s_lb[nB + base + lane_prefix(bal)] = (uint16_t)li;
      nB += tot;
      __syncthreads();
    }

    // S3: the full mixture with the confidence-driven learning rate.
    for (int i = tid; i < nB; i += kNT) {
      const int li = s_lb[i];
      const int64_t p = tile0 + li;
      float xx[C];
#pragma unroll
      for (int c = 0; c < C; ++c) xx[c] = s_x[li * C + c];
      const float ae = kp.alpha * (1.0f - kp.kappa * s_conf[li]);
      Mix<C, K> m;
      rec_load<C, K>(b.gmm + p * R, m);
      int l, mp;
      mix_step<C, K>(m, xx, ae, kp, l, mp);
      rec_store<C, K>(b.gmm + p * R, m);
      uint8_t res = (uint8_t)((3 << 2) | (l ? 1 : 0));
      if (!l) {
        // background from the mixture: the running average takes the matched
        // component (the transition update of the active level)
        float sm[C], sv = m.var[0];
#pragma unroll
        for (int c = 0; c < C; ++c) sm[c] = m.mu[0][c];
#pragma unroll
        for (int k = 1; k < K; ++k) {
          if (mp == k) {
            sv = m.var[k];
#pragma unroll
            for (int c = 0; c < C; ++c) sm[c] = m.mu[k][c];
          }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) s_rg[li * (C + 1) + c] = sm[c];
        s_rg[li * (C + 1) + C] = sv;
        res |= 2;
      }
      s_res[li] = res;
    }
    __syncthreads();

    uint8_t *mk = fr.mask ? fr.mask + (int64_t)f * fr.mstride : nullptr;
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c3bg = 0, cfg = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int64_t p = tile0 + j * kNT + tid;
      const int li = j * kNT + tid;
      if (surv[j]) {
        const uint8_t r = s_res[li];
        lab[j] = (r & 1) != 0;
        st[j] = r >> 2;
        if (r & 2) {
#pragma unroll
          for (int c = 0; c < C; ++c) rmu[j][c] = s_rg[li * (C + 1) + c];
          rvar[j] = s_rg[li * (C + 1) + C];
          dirty[j] = true;
        }
      }
      if (valid[j]) {
        if (mk) mk[p] = lab[j] ? 255 : 0;
#pragma unroll
        for (int c = 0; c < C; ++c) xp[j][c] = x[j][c];
      }
      c0 += (uint32_t)__popcll(__ballot(st[j] == 0));
      c1 += (uint32_t)__popcll(__ballot(st[j] == 1));
      c2 += (uint32_t)__popcll(__ballot(st[j] == 2));
      c3 += (uint32_t)__popcll(__ballot(st[j] == 3));
      c3bg += (uint32_t)__popcll(__ballot(st[j] == 3 && !lab[j]));
      cfg += (uint32_t)__popcll(__ballot(valid[j] && lab[j]));
    }
    if (lane == 0) {
      uint32_t *sp = &s_stat[f & 1][0];
      atomicAdd(sp + 0, c0);
      atomicAdd(sp + 1, c1);
      atomicAdd(sp + 2, c2);
      atomicAdd(sp + 3, c3);
      atomicAdd(sp + 4, c3bg);
      atomicAdd(sp + 5, cfg);
    }
  }
  __syncthreads();
  if (tid == 0 && fr.nframes > 0 && fr.partials) {
    const int f = fr.nframes - 1;
    uint32_t *dst = fr.partials + ((int64_t)f * fr.nslots + blockIdx.x) * kStat;
#pragma unroll
    for (int k = 0; k < kStat; ++k) dst[k] = s_stat[f & 1][k];
  }

#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int64_t p = tile0 + j * kNT + tid;
    if (valid[j]) {
      if (dirty[j]) {
        float *rg = b.rga + p * RG;
#pragma unroll
        for (int c = 0; c < C; ++c) rg[c] = rmu[j][c];
        rg[C] = rvar[j];
      }
      store_px<C, F32>(b.prev, p, xp[j]);
    }
    const unsigned long long bal = __ballot(lab[j]);
    const int64_t w0 = tile0 + j * kNT + wave * 64;
    if (lane == 0 && w0 < b.P) b.labels[w0 >> 6] = bal;
  }
}

// ============================================================================
// Plain Stauffer-Grimson baseline: every pixel runs the mixture step every
// frame (alpha fixed), one pixel per thread, state in registers across the
// frames of the launch, 64-pixel field-major record groups.
template <int C, int K, bool F32>
__global__ __launch_bounds__(kNT) void k_gmm(Buffers b, Frames fr, KParams kp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const bool valid = p < b.P;
  Mix<C, K> m;
  float x[C];
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = 0.0f;
  if (valid) grp_load<C, K>(b.gmm, p, m);
  bool lab = false;
  for (int f = 0; f < fr.nframes; ++f) {
    if (valid) {
      load_px<C, F32>(frame_ptr<C, F32>(fr.x, fr.stride, f), p, x);
      int l, mp;
      mix_step<C, K>(m, x, kp.alpha, kp, l, mp);
      lab = l != 0;
      if (fr.mask) fr.mask[(int64_t)f * fr.mstride + p] = lab ? 255 : 0;
    }
    if (fr.partials) {
      const uint32_t nv = (uint32_t)__popcll(__ballot(valid));
      const uint32_t nf = (uint32_t)__popcll(__ballot(valid && lab));
      if (lane == 0) {
        uint32_t *dst =
            fr.partials + ((int64_t)f * fr.nslots + (int64_t)blockIdx.x * kNW + wave) * kStat;
        dst[0] = 0u;
        dst[1] = 0u;
        dst[2] = 0u;
        dst[3] = nv;
        dst[4] = nv - nf;
        dst[5] = nf;
        dst[6] = 0u;
        dst[7] = 0u;
      }
    }
  }
  if (valid) {
    grp_store<C, K>(b.gmm, p, m);
    if (fr.nframes > 0) store_px<C, F32>(b.prev, p, x);
  }
  const unsigned long long bal = __ballot(lab);
  const int64_t w0 = p - lane;
  if (fr.nframes > 0 && lane == 0 && w0 < b.P) b.labels[w0 >> 6] = bal;
}

}  // namespace

// ---- launchers ---------------------------------------------------------------
#define COG_K_CASES(M, ...) \
  switch (K) {              \
    case 1: M(1, __VA_ARGS__); break; \
    case 2: M(2, __VA_ARGS__); break; \
    case 3: M(3, __VA_ARGS__); break; \
    case 4: M(4, __VA_ARGS__); break; \
    case 5: M(5, __VA_ARGS__); break; \
    case 6: M(6, __VA_ARGS__); break; \
    case 7: M(7, __VA_ARGS__); break; \
    case 8: M(8, __VA_ARGS__); break; \
    default: return hipErrorInvalidValue; \
  }

static unsigned grid_for(int64_t P, int tile) { return (unsigned)((P + tile - 1) / tile); }

hipError_t launch_train(int C, int K, bool f32in, bool prior, bool aos, const Buffers &b,
                        const void *frames, int64_t stride, int n, const KParams &kp,
                        hipStream_t s) {
  const unsigned g = grid_for(b.P, kNT);
#define COG_TRAIN(KK, CC, FF)                                                                  \
  hipLaunchKernelGGL((k_train<CC, KK, FF>), dim3(g), dim3(kNT), 0, s, b, frames, stride, n, kp, \
                     prior ? 1 : 0, aos ? 1 : 0)
  if (C == 3 && !f32in) { COG_K_CASES(COG_TRAIN, 3, false) }
  else if (C == 3 && f32in) { COG_K_CASES(COG_TRAIN, 3, true) }
  else if (C == 1 && !f32in) { COG_K_CASES(COG_TRAIN, 1, false) }
  else if (C == 1 && f32in) { COG_K_CASES(COG_TRAIN, 1, true) }
  else return hipErrorInvalidValue;
#undef COG_TRAIN
  return hipGetLastError();
}

hipError_t launch_cascade(int C, int K, bool f32in, int ppt, const Buffers &b, const Frames &fr,
                          const KParams &kp, hipStream_t s) {
  const unsigned g = grid_for(b.P, kNT * ppt);
#define COG_CASC(KK, CC, FF, PP) \
  hipLaunchKernelGGL((k_cascade<CC, KK, FF, PP>), dim3(g), dim3(kNT), 0, s, b, fr, kp)
#define COG_CASC_PPT(CC, FF)                                        \
  switch (ppt) {                                                   \
    case 1: { COG_K_CASES(COG_CASC, CC, FF, 1) } break;            \
    case 2: { COG_K_CASES(COG_CASC, CC, FF, 2) } break;            \
    case 4: { COG_K_CASES(COG_CASC, CC, FF, 4) } break;            \
    default: return hipErrorInvalidValue;                          \
  }
  if (C == 3 && !f32in) { COG_CASC_PPT(3, false) }
  else if (C == 3 && f32in) { COG_CASC_PPT(3, true) }
  else if (C == 1 && !f32in) { COG_CASC_PPT(1, false) }
  else if (C == 1 && f32in) { COG_CASC_PPT(1, true) }
  else return hipErrorInvalidValue;
#undef COG_CASC_PPT
#undef COG_CASC
  return hipGetLastError();
}

hipError_t launch_gmm(int C, int K, bool f32in, const Buffers &b, const Frames &fr,
                      const KParams &kp, hipStream_t s) {
  const unsigned g = grid_for(b.P, kNT);
#define COG_GMM(KK, CC, FF) \
  hipLaunchKernelGGL((k_gmm<CC, KK, FF>), dim3(g), dim3(kNT), 0, s, b, fr, kp)
  if (C == 3 && !f32in) { COG_K_CASES(COG_GMM, 3, false) }
  else if (C == 3 && f32in) { COG_K_CASES(COG_GMM, 3, true) }
  else if (C == 1 && !f32in) { COG_K_CASES(COG_GMM, 1, false) }
  else if (C == 1 && f32in) { COG_K_CASES(COG_GMM, 1, true) }
  else return hipErrorInvalidValue;
#undef COG_GMM
  return hipGetLastError();
}

}  // namespace cog
