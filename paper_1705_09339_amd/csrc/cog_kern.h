// Kernel templates of the Cascade-of-Gaussians background subtractor
// (arXiv 1705.09339) for gfx950: prior training, the fused rejection cascade,
// the batched tick and the plain mixture baseline, with their launchers
// templated on the mixture size K.  Each K is instantiated in a translation
// unit of its own (cog_inst_k*.hip), so the library builds in parallel.
//
// Numerics: every floating-point expression below is evaluated as written,
// one binary32 round-to-nearest-even operation at a time (the library is
// built with -ffp-contract=off, IEEE denormals and correctly rounded
// division), so the discrete decisions of the method -- component match,
// background set, rank order, cascade gates -- are reproducible bit for bit.
// There are no transcendental functions on the per-frame path; the rank key
// w/sigma is compared as w_a^2 sigma_b^2 > w_b^2 sigma_a^2.
#pragma once

#include "cog_device.h"

namespace cog {
namespace {

// ----------------------------------------------------------------------------
// a / d correctly rounded from y = 1/d correctly rounded: q = a y, then twice
// q <- q + (a - d q) y with the residual formed by a fused multiply-add.  The
// first correction leaves q within one unit in the last place of a / d, so
// its residual is exact, and the second returns the correctly rounded
// quotient (Markstein's theorem).  It holds when |d| is in [2^-20, 2^20] and
// a is +0 or |a| is in [2^-100, 2^60]: then no residual loses bits to
// underflow and nothing overflows.  Callers check that range (or know it) and
// divide outside it; one reciprocal then serves every quotient by d.
__device__ __forceinline__ float quot_recip(float a, float d, float y) {
  const float q0 = a * y;
  const float q1 = __builtin_fmaf(__builtin_fmaf(-d, q0, a), y, q0);
  return __builtin_fmaf(__builtin_fmaf(-d, q1, a), y, q1);
}

// Bit patterns of the range bounds above (binary32, positive).
constexpr uint32_t kDivisorLo = 0x35800000u;  // 2^-20
constexpr uint32_t kDivisorHi = 0x49800000u;  // 2^20
constexpr uint32_t kDividendLo = 0x0d800000u; // 2^-100
constexpr uint32_t kDividendHi = 0x5d800000u; // 2^60

__device__ __forceinline__ bool divisor_in_range(float d) {
  return __float_as_uint(d) - kDivisorLo <= kDivisorHi - kDivisorLo;  // positive d only
}

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

// Background set B: the smallest b whose cumulative weight exceeds T (K when
// none does).  Written as a running minimum over the candidates b + 1, which
// increase with b, so it compiles to selects rather than branches.
template <int C, int K>
__device__ __forceinline__ int mix_bgset(const Mix<C, K> &s, float T) {
  float cum = 0.0f;
  int B = K;
#pragma unroll
  for (int b = 0; b < K; ++b) {
    cum = cum + s.w[b];
    const int cand = cum > T ? b + 1 : K;
    B = cand < B ? cand : B;
  }
  return B;
}

// One mixture step (§2, the update equation under "Scene Prior"):
// classify against the pre-update ranks, w <- (1-a)w + aM, the matched
// component's mean and variance move with rho = a / w_m, an unmatched value
// replaces the last-ranked slot, weights are renormalised and the slots are
// re-ranked by w/sigma (stable).  Returns the label (1 = foreground) and the
// matched slot's rank after the re-sort (-1 when nothing matched).  LABEL
// false skips the background set and returns label 0, for warm-up frames
// whose label is not kept; the state update is the same.
template <int C, int K, bool LABEL = true>
__device__ __forceinline__ void mix_step(Mix<C, K> &s, const float (&x)[C], float ae,
                                         const KParams &kp, int &label, int &mpost) {
  const int B = LABEL ? mix_bgset<C, K>(s, kp.T) : K;
  // first matching rank: every distance is evaluated (no short-circuit) and
  // the scan runs from the last rank down, so the lowest hit wins as a select
  int m = -1;
#pragma unroll
  for (int k = K - 1; k >= 0; --k) {
    float d2 = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float d = x[c] - s.mu[k][c];
      d2 = d2 + d * d;
    }
    const bool hit = (s.w[k] > 0.0f) & (d2 <= kp.lam2 * s.var[k]);
    m = hit ? k : m;
  }
  label = LABEL ? ((m >= 0 && m < B) ? 0 : 1) : 0;

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
  // the K quotients w_k / S share one reciprocal when S and every w_k are in
  // quot_recip's range: the smallest (pattern - 1) skips zeros (+0 wraps to
  // the top), the largest pattern rejects negatives, infinities and NaNs
  uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t u = __float_as_uint(s.w[k]);
    lo = min(lo, u - 1u);
    hi = max(hi, u);
  }
  if (divisor_in_range(S) && lo >= kDividendLo - 1u && hi <= kDividendHi) {
    const float y = 1.0f / S;
#pragma unroll
    for (int k = 0; k < K; ++k) s.w[k] = quot_recip(s.w[k], S, y);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) s.w[k] = s.w[k] / S;
  }

  // Re-rank by w/sigma: stable insertion sort with early exit, pass i moving
  // slot i toward the front while it ranks strictly above its predecessor.
  // If no adjacent pair is out of order no pass exchanges anything, so the
  // passes run only in lanes with an adjacent inversion.  A lane stops a pass
  // at its first comparison without exchange, exactly as the sequential sort;
  // the wave leaves the pass once none of its lanes is still moving.
  int mp = m;
  bool inverted = false;
#pragma unroll
  for (int j = 1; j < K; ++j)
    inverted |= (s.w[j] * s.w[j]) * s.var[j - 1] > (s.w[j - 1] * s.w[j - 1]) * s.var[j];
  if (inverted) {
#pragma unroll
    for (int i = 1; i < K; ++i) {
      bool mv = true;
#pragma unroll
      for (int j = i; j > 0; --j) {
        const float lhs = (s.w[j] * s.w[j]) * s.var[j - 1];
        const float rhs = (s.w[j - 1] * s.w[j - 1]) * s.var[j];
        mv = mv && lhs > rhs;
        if (__ballot(mv) == 0ull) break;
        if (mv) {
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
  }
  mpost = mp;
}

// ---- mixture record layouts ------------------------------------------------
// Cascade: one record of rec_floats(C,K) floats per pixel, {w[K], var[K],
// mu[K][C]}, 16-byte aligned, so a lone survivor reads one or two lines.
template <int C, int K>
__device__ __forceinline__ void rec_load(const float *rec, Mix<C, K> &s) {
  constexpr int R = (mix_floats(C, K) + 3) & ~3;  // the used 16-byte words only
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

// Field i of a record: w[K], var[K], mu[K][C], then zero padding (i is a
// compile-time index once the callers' loops are unrolled).
template <int C, int K>
__device__ __forceinline__ float rec_field(const Mix<C, K> &s, int i) {
  if (i < K) return s.w[i];
  if (i < 2 * K) return s.var[i - K];
  if (i < mix_floats(C, K)) return s.mu[(i - 2 * K) / C][(i - 2 * K) % C];
  return 0.0f;
}

template <int C, int K>
__device__ __forceinline__ void rec_store(float *rec, const Mix<C, K> &s) {
  constexpr int R = (mix_floats(C, K) + 3) & ~3;  // up to the last used 16-byte word
  float4 *r4 = reinterpret_cast<float4 *>(rec);
#pragma unroll
  for (int i = 0; i < R / 4; ++i)
    r4[i] = make_float4(rec_field(s, 4 * i), rec_field(s, 4 * i + 1), rec_field(s, 4 * i + 2),
                        rec_field(s, 4 * i + 3));
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


// Raw input registers: the load result is kept untouched until the frame it
// belongs to is processed, so a prefetch issued one frame early is not waited
// for before its first real use.
template <bool F32>
struct RawT { using type = uint32_t; };
template <>
struct RawT<true> { using type = float; };

template <int C, bool F32>
__device__ __forceinline__ void raw_load(const void *base, int64_t p,
                                         typename RawT<F32>::type (&r)[C]) {
  if constexpr (F32) {
    const float *q = static_cast<const float *>(base) + p * C;
#pragma unroll
    for (int c = 0; c < C; ++c) r[c] = __builtin_nontemporal_load(q + c);
  } else {
    const uint8_t *q = static_cast<const uint8_t *>(base) + p * C;
#pragma unroll
    for (int c = 0; c < C; ++c) r[c] = (uint32_t)__builtin_nontemporal_load(q + c);
  }
}

template <int C, bool F32>
__device__ __forceinline__ void raw_to_float(const typename RawT<F32>::type (&r)[C], float (&x)[C]) {
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = (float)r[c];
}


// u8 input, one wave per 64 consecutive pixels: the wave's 64*C bytes are
// read as the dwords of the 4-byte-aligned window that covers them (lane i
// loads dword i), and each lane later picks its C bytes out with a lane
// permute.  Aligned dwords never straddle a page, so the at most 3 bytes read
// beyond either end of the run cannot fault.  npx >= 1 valid pixels.
template <int C>
__device__ __forceinline__ uint32_t u8win_load(const uint8_t *frame, int64_t first_px, int npx,
                                               int lane) {
  const uint8_t *start = frame + first_px * C;
  const int mis = (int)(reinterpret_cast<uintptr_t>(start) & 3);
  // derived by pointer arithmetic so that the load stays a global (not flat) load
  const uint32_t *al = reinterpret_cast<const uint32_t *>(start - mis);
  const int nd = (mis + npx * C + 3) >> 2;
  return __builtin_nontemporal_load(al + (lane < nd ? lane : nd - 1));
}

template <int C>
__device__ __forceinline__ void u8win_extract(uint32_t raw, const uint8_t *frame, int64_t first_px,
                                              int lane, float (&x)[C]) {
  const int mis = (int)(reinterpret_cast<uintptr_t>(frame + first_px * C) & 3);
  const int o = mis + C * lane;
  const int w0 = o >> 2;
  const uint32_t d0 = (uint32_t)__builtin_amdgcn_ds_bpermute(w0 << 2, (int)raw);
  if constexpr (C == 1) {
    x[0] = (float)((d0 >> (8 * (o & 3))) & 0xffu);
  } else {
    const uint32_t d1 = (uint32_t)__builtin_amdgcn_ds_bpermute((w0 + 1) << 2, (int)raw);
    const uint32_t win = __builtin_amdgcn_alignbyte(d1, d0, (uint32_t)(o & 3));
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = (float)((win >> (8 * c)) & 0xffu);
  }
}


// Block-staged input for one wave of 64 consecutive pixels.  The wave's
// window of a frame is 64*C input values; each lane loads NDW dwords of it
// (u8: lane i loads dword i of the 4-byte-aligned window, at most 49 dwords;
// f32: dwords i, i+64, ...).  Every NB frames the windows of the next NB
// frames are requested into registers and the ones requested a block
// earlier are copied into an LDS ring, so a frame's input is an LDS read and
// the global-memory wait is paid once per NB frames, on loads issued NB
// frames before.  Slots past the last frame are not loaded (and never read).
template <int C, bool F32, int NB>
struct InStage {
  static constexpr int NDW = F32 ? C : 1;
  uint32_t r[NB][NDW];

  __device__ __forceinline__ void issue(const void *x, int64_t stride, int nframes, int fb,
                                        int64_t tile0, int npx, int lane) {
#pragma unroll
    for (int kk = 0; kk < NB; ++kk) {
      const int ff = fb + kk;
      if (ff >= nframes) break;  // wave-uniform
      const void *xf = frame_ptr<C, F32>(x, stride, ff);
      if constexpr (F32) {
        const uint32_t *base = reinterpret_cast<const uint32_t *>(xf) + tile0 * C;
        const int nd = npx * C;
#pragma unroll
        for (int d = 0; d < NDW; ++d) {
          const int i = lane + 64 * d;
          r[kk][d] = __builtin_nontemporal_load(base + (i < nd ? i : nd - 1));
        }
      } else {
        r[kk][0] = u8win_load<C>(static_cast<const uint8_t *>(xf), tile0, npx, lane);
      }
    }
  }

  __device__ __forceinline__ void commit(uint32_t *s, int lane) const {
#pragma unroll
    for (int kk = 0; kk < NB; ++kk)
#pragma unroll
      for (int d = 0; d < NDW; ++d) s[(kk * NDW + d) * 64 + lane] = r[kk][d];
  }

  // value of this lane's pixel in slot k; mis = the frame's run misalignment
  static __device__ __forceinline__ void read_mis(const uint32_t *s, int k, int mis, int lane,
                                                  float (&x)[C]) {
    if constexpr (F32) {
      const float *fs = reinterpret_cast<const float *>(s + k * NDW * 64);
#pragma unroll
      for (int c = 0; c < C; ++c) x[c] = fs[C * lane + c];
    } else {
      const uint8_t *bs = reinterpret_cast<const uint8_t *>(s + k * 64);
#pragma unroll
      for (int c = 0; c < C; ++c) x[c] = (float)bs[mis + C * lane + c];
    }
  }

  // value of this lane's pixel in slot k (frame xf of the ring)
  static __device__ __forceinline__ void read(const uint32_t *s, int k, const void *xf,
                                              int64_t tile0, int lane, float (&x)[C]) {
    if constexpr (F32) {
      const float *fs = reinterpret_cast<const float *>(s + k * NDW * 64);
#pragma unroll
      for (int c = 0; c < C; ++c) x[c] = fs[C * lane + c];
    } else {
      const uint8_t *bs = reinterpret_cast<const uint8_t *>(s + k * 64);
      const int mis =
          (int)(reinterpret_cast<uintptr_t>(static_cast<const uint8_t *>(xf) + tile0 * C) & 3);
#pragma unroll
      for (int c = 0; c < C; ++c) x[c] = (float)bs[mis + C * lane + c];
    }
  }
};


// Compiler-level ordering of LDS accesses between the lanes of one wave (the
// hardware executes a wave's LDS instructions in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// max_c |x_c - xp_c| (a NaN difference is skipped, as by the comparison form)
template <int C>
__device__ __forceinline__ float frame_delta(const float (&x)[C], const float (&xp)[C]) {
  float dl = 0.0f;
#pragma unroll
  for (int c = 0; c < C; ++c) dl = fmaxf(dl, fabsf(x[c] - xp[c]));
  return dl;
}

__device__ __forceinline__ int lane_prefix(unsigned long long bal) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
}


// S2 (§2 "Confidence Measure", "Cascade of Gaussians CoG"): the scene-prior
// probability of x from the pixel's u8 KDE table (channels independent, so
// the product of the per-channel entries), then C = a P + b D + g M with the
// weights a, b, g from the training residue histogram, D the frame-difference
// similarity and M the distance to the running average; a is dropped when P
// is below p_null (prior nullified).  rec is the pixel's prior record:
// t[C][16] u8, then a, b, g as f32.
template <int C, bool F32>
__device__ __forceinline__ float confidence(const uint8_t *rec, const float (&x)[C], float dl,
                                            float dr2, float var_r, const KParams &kp) {
  uint32_t prod = 1u;
#pragma unroll
  for (int c = 0; c < C; ++c) prod = prod * (uint32_t)rec[c * kBins + (quant<F32>(x[c], kp) >> 4)];
  // prod is an integer in [0, 255^C] and the divisor a constant whose
  // reciprocal is rounded at compile time: dividends of at least 1 and
  // quotients in [2^-24, 1] keep quot_recip exact (all 255^C + 1 cases agree
  // with the division, checked exhaustively)
  constexpr float kTop = C == 3 ? 16581375.0f : 255.0f;
  const float ph = quot_recip((float)prod, kTop, 1.0f / kTop);
  const float *abg = reinterpret_cast<const float *>(rec + C * kBins);
  float a = abg[0];
  const float bw = abg[1];
  const float g = abg[2];
  if (ph < kp.p_null) a = 0.0f;
  // u8 input: dl is an integer in [0, 255], in range whenever res_e2 is
  // (inv_res_e2 != 0, a uniform branch)
  float dh;
  if (!F32 && kp.inv_res_e2 != 0.0f)
    dh = 1.0f - quot_recip(dl, kp.res_e2, kp.inv_res_e2);
  else
    dh = 1.0f - dl / kp.res_e2;
  dh = dh < 0.0f ? 0.0f : dh;
  float mh = 1.0f - dr2 / (kp.lam_m2 * var_r);
  mh = mh < 0.0f ? 0.0f : mh;
  return (a * ph + bw * dh) + g * mh;
}

// ============================================================================
// Training phase: each pixel's N training frames are walked once for
//  - integer KDE bin masses acc[c][b] += W[b][q(x)] (weights staged in LDS,
//    level-major so one level's 16 weights are two 16-byte reads),
//  - the residue histogram over max_c |x_j - x_{j-1}|,
//  - the mixture warm-up (initialised from frame 0, stepped on 1..N-1).
// Then the max-normalised u8 table, counts, mixture, running average (from
// the dominant mode), previous frame and label are written once.  The
// baseline mixture trains only the warm-up.
// floor((255 a + floor(d / 2)) / d) for 0 <= a <= d, d > 0, exactly.  The
// quotient is at most 255: a binary32 estimate is within one of it (its
// relative error is below 2^-22), and two exact 64-bit comparisons correct it,
// instead of a full 64-bit integer division.
__device__ __forceinline__ uint32_t round_ratio255(uint32_t a, uint32_t d) {
  const uint64_t num = 255ull * a + (d >> 1);
  int32_t q = (int32_t)((float)num / (float)d);
  q = q < 0 ? 0 : (q > 255 ? 255 : q);
  if ((uint64_t)(uint32_t)q * d > num) --q;
  if ((uint64_t)(uint32_t)(q + 1) * d <= num) ++q;
  return (uint32_t)q;
}

// Grouping key of a temporal variance (§2 "Clustering Similar Background"):
// var = Q/n - (S/n)^2 from the warm-up sums, clamped at 0, as the top 16
// bits of its binary32 pattern (a piecewise-linear log2 scale).
__device__ __forceinline__ uint32_t var_key(float S, float Q, float n) {
  const float m = S / n;
  float var = Q / n - m * m;
  var = var > 0.0f ? var : 0.0f;
  return __float_as_uint(var) >> 16;
}

// One shared parameter set per group (§2 "Clustering Similar Background"):
// the stored running-average variance carries the pixel's group flag in its
// sign bit.  When set, the magnitude is the group's shared variance, which
// the pixel uses and never adapts.  Every use takes the magnitude (a free
// source modifier); an update keeps a shared value as it is.
__device__ __forceinline__ bool rvar_shared(float stored) {
  return (int32_t)__float_as_uint(stored) < 0;
}

// Warm-up of the plain mixture baseline: one thread per pixel steps its
// mixture over the N training frames and stores it in the grouped layout.
template <int C, int K, bool F32>
__global__ __launch_bounds__(kNT) void k_train(Buffers b, const void *frames, int64_t stride,
                                               int n, KParams kp, int64_t p0, int64_t p1) {
  const int lane = threadIdx.x & 63;
  const int64_t p = p0 + (int64_t)blockIdx.x * kNT + threadIdx.x;
  const bool valid = p < p1;
  bool lab = false;
  if (valid) {
    float x[C], xp[C], xn[C];
    Mix<C, K> m;
    load_px<C, F32>(frames, p, x);
    mix_init<C, K>(m, x, kp.var_init);
    // the next frame's value is requested one frame ahead, so its latency
    // overlaps the current frame's work
#pragma unroll
    for (int c = 0; c < C; ++c) xp[c] = x[c];
    if (n > 1) load_px<C, F32>(frame_ptr<C, F32>(frames, stride, 1), p, xn);
    // frames 1..n-2 without the label (only the last frame's is kept), then
    // frame n-1 with it
    for (int j = 1; j + 1 < n; ++j) {
#pragma unroll
      for (int c = 0; c < C; ++c) x[c] = xn[c];
      load_px<C, F32>(frame_ptr<C, F32>(frames, stride, j + 1), p, xn);
      int l, mp;
      mix_step<C, K, false>(m, x, kp.alpha, kp, l, mp);
#pragma unroll
      for (int c = 0; c < C; ++c) xp[c] = x[c];
    }
    if (n > 1) {
#pragma unroll
      for (int c = 0; c < C; ++c) x[c] = xn[c];
      int l, mp;
      mix_step<C, K, true>(m, x, kp.alpha, kp, l, mp);
      lab = l != 0;
#pragma unroll
      for (int c = 0; c < C; ++c) xp[c] = x[c];
    }
    grp_store<C, K>(b.gmm, p, m);
    store_px<C, F32>(b.prev, p, xp);
  }
  const unsigned long long bal = __ballot(lab);
  const int64_t w0 = p - lane;
  if (lane == 0 && w0 < b.P) b.labels[w0 >> 6] = bal;
}

// Training of the cascade (§2 "Scene Prior", "Cascade of Gaussians CoG") in
// two wave roles: a workgroup covers kTrainPx pixels with twice as many
// threads.  Its first waves accumulate the kernel-density bins and the
// residue counts and write the prior record; its other waves run the mixture
// warm-up over the same pixels and write the mixture, running average,
// previous value, label and grouping keys.  The two roles read the same
// frames and run concurrently.  Each holds only its own accumulators (the
// 48 bin accumulators, or the mixture), so a thread needs about half the
// registers of one that holds both and more than twice as many waves stay
// resident.
constexpr int kTrainPx = 128;

// The prior record of a trained pixel from its bin masses acc and residue
// counts: the max-normalised u8 table, the confidence weights and the counts.
template <int C>
__device__ __forceinline__ void store_prior(const Buffers &b, int64_t p,
                                            const uint32_t (&acc)[C][kBins], uint32_t cnt0,
                                            uint32_t cnt1, uint32_t cnt2, const KParams &kp) {
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
      const uint32_t tq = amax ? round_ratio255(acc[c][q], amax) : 0u;
      const int byte = c * kBins + q;
      words[byte >> 2] |= (tq & 0xffu) << (8 * (byte & 3));
    }
  }
  // confidence weights a, b, g = counts / (N - 1), divided once here
  words[(C * kBins) / 4] = __float_as_uint((float)cnt0 / kp.nm1);
  words[(C * kBins) / 4 + 1] = __float_as_uint((float)cnt1 / kp.nm1);
  words[(C * kBins) / 4 + 2] = __float_as_uint((float)cnt2 / kp.nm1);
  *reinterpret_cast<uint2 *>(b.cnt + p * 4) =
      make_uint2((cnt0 & 0xffffu) | (cnt1 << 16), cnt2 & 0xffffu);
  uint4 *dst = reinterpret_cast<uint4 *>(b.prior + p * PB);
#pragma unroll
  for (int i = 0; i < PB / 16; ++i)
    dst[i] = make_uint4(words[4 * i], words[4 * i + 1], words[4 * i + 2], words[4 * i + 3]);
}

// The mixture role of a training workgroup: the warm-up (initialised from
// frame 0, stepped on 1..N-1) and the grouping sums of pixel p, then the
// mixture record, running average, keys, previous value and label word.
template <int C, int K, bool F32>
__device__ __forceinline__ void train_mixture_role(const Buffers &b, const void *frames,
                                                   int64_t stride, int n, const KParams &kp,
                                                   int64_t p, bool valid, int lane) {
  bool lab = false;
  if (valid) {
    // grouping features: sums over the warm-up of the dominant component's
    // adapted variance and weight and of their squares
    float sv = 0.0f, qv = 0.0f, sw = 0.0f, qw = 0.0f;
    float x[C], xp[C], xn[C];
    Mix<C, K> m;
    load_px<C, F32>(frames, p, x);
    mix_init<C, K>(m, x, kp.var_init);
#pragma unroll
    for (int c = 0; c < C; ++c) xp[c] = x[c];
    if (n > 1) load_px<C, F32>(frame_ptr<C, F32>(frames, stride, 1), p, xn);
    // frames 1..n-2 without the label (only the last frame's is kept), then
    // frame n-1 with it
    for (int j = 1; j + 1 < n; ++j) {
#pragma unroll
      for (int c = 0; c < C; ++c) x[c] = xn[c];
      load_px<C, F32>(frame_ptr<C, F32>(frames, stride, j + 1), p, xn);
      int l, mp;
      mix_step<C, K, false>(m, x, kp.alpha, kp, l, mp);
      sv = sv + m.var[0];
      qv = qv + m.var[0] * m.var[0];
      sw = sw + m.w[0];
      qw = qw + m.w[0] * m.w[0];
#pragma unroll
      for (int c = 0; c < C; ++c) xp[c] = x[c];
    }
    if (n > 1) {
#pragma unroll
      for (int c = 0; c < C; ++c) x[c] = xn[c];
      int l, mp;
      mix_step<C, K, true>(m, x, kp.alpha, kp, l, mp);
      lab = l != 0;
      sv = sv + m.var[0];
      qv = qv + m.var[0] * m.var[0];
      sw = sw + m.w[0];
      qw = qw + m.w[0] * m.w[0];
#pragma unroll
      for (int c = 0; c < C; ++c) xp[c] = x[c];
    }
    constexpr int RG = rga_floats(C);
    float *rg = b.rga + p * RG;
#pragma unroll
    for (int c = 0; c < C; ++c) rg[c] = m.mu[0][c];
    rg[C] = m.var[0];
    b.sat[p] = 0;  // no confident frame yet (sampling)
    b.gkey[p] = make_uint2(var_key(sv, qv, kp.nm1), var_key(sw, qw, kp.nm1));
    rec_store<C, K>(b.gmm + p * rec_floats(C, K), m);
    store_px<C, F32>(b.prev, p, xp);
  }
  const unsigned long long bal = __ballot(lab);
  const int64_t w0 = p - lane;
  if (lane == 0 && w0 < b.P) b.labels[w0 >> 6] = bal;
}

// Widened weights: the table holds each weight in 32 bits, so that one
// 64-bit add accumulates two adjacent bins (neither half can carry:
// n * 65535 < 2^32 for n <= 65536).  Used for u8 input with K <= 7, where
// the mixture role leaves room for it at 7 waves per SIMD; f32 input (whose
// quantisation needs registers) and K = 8 keep the 16-bit table and one add
// per bin.
template <int K, bool F32>
constexpr bool train_wide_table() { return !F32 && K <= 7; }
// Minimum waves per SIMD asked of the compiler (1: no constraint).
template <int K, bool F32>
constexpr int train_prior_waves() { return train_wide_table<K, F32>() ? 7 : 1; }

template <int C, int K, bool F32>
__global__ __launch_bounds__(2 * kTrainPx)
__attribute__((amdgpu_waves_per_eu(train_prior_waves<K, F32>()))) void k_train_prior(
    Buffers b, const void *frames, int64_t stride, int n, KParams kp, int64_t p0, int64_t p1) {
  constexpr bool WIDE = train_wide_table<K, F32>();
  constexpr int TW = WIDE ? 256 * kBins / 4 : 256 * kBins / 8;  // uint4 words
  __shared__ uint4 s_w[TW];
  // chunk-major in LDS: chunk h of level v at s_w[h * 256 + v], so lanes whose
  // levels lie within a few steps of each other read different banks
  constexpr int NCH = TW / 256;  // 16-byte chunks per level
  for (int i = threadIdx.x; i < TW; i += 2 * kTrainPx) {
    const int v = i / NCH, h = i % NCH;
    if constexpr (WIDE) {
      const uint2 w = reinterpret_cast<const uint2 *>(b.kdew)[i];
      s_w[h * 256 + v] = make_uint4(w.x & 0xffffu, w.x >> 16, w.y & 0xffffu, w.y >> 16);
    } else {
      s_w[h * 256 + v] = reinterpret_cast<const uint4 *>(b.kdew)[i];
    }
  }
  __syncthreads();

  const bool prior_role = threadIdx.x < kTrainPx;  // wave-uniform
  const int t = prior_role ? threadIdx.x : threadIdx.x - kTrainPx;
  const int lane = t & 63;
  const int64_t p = p0 + (int64_t)blockIdx.x * kTrainPx + t;
  const bool valid = p < p1;
  if (!prior_role) {
    train_mixture_role<C, K, F32>(b, frames, stride, n, kp, p, valid, lane);
    return;
  }
  if (!valid) return;
  // wide: bins 2q (low half) and 2q + 1 (high half) of acc2[c][q]
  uint64_t acc2[C][WIDE ? kBins / 2 : 1];
  uint32_t acc[C][kBins];
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int q = 0; q < (WIDE ? kBins / 2 : 1); ++q) acc2[c][q] = 0u;
#pragma unroll
    for (int q = 0; q < kBins; ++q) acc[c][q] = 0u;
  }
  uint32_t cnt0 = 0, cnt1 = 0, cnt2 = 0;
  float x[C], xp[C], xn[C];
  load_px<C, F32>(frames, p, x);
  if (n > 1) load_px<C, F32>(frame_ptr<C, F32>(frames, stride, 1), p, xn);
  for (int j = 0; j < n; ++j) {
    if (j >= 1) {
#pragma unroll
      for (int c = 0; c < C; ++c) x[c] = xn[c];
      if (j + 1 < n) load_px<C, F32>(frame_ptr<C, F32>(frames, stride, j + 1), p, xn);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int v = quant<F32>(x[c], kp);
      if constexpr (WIDE) {
#pragma unroll
        for (int h = 0; h < kBins / 4; ++h) {
          const uint4 w4 = s_w[h * 256 + v];
          acc2[c][2 * h] += (uint64_t)w4.x | ((uint64_t)w4.y << 32);
          acc2[c][2 * h + 1] += (uint64_t)w4.z | ((uint64_t)w4.w << 32);
        }
      } else {
        const uint4 lo = s_w[v], hi = s_w[256 + v];
        const uint32_t wd[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          acc[c][2 * q] += wd[q] & 0xffffu;
          acc[c][2 * q + 1] += wd[q] >> 16;
        }
      }
    }
    if (j >= 1) {
      const float dl = frame_delta<C>(x, xp);
      // residue bins [0, e1), [e1, e2), [e2, inf) counted without branches
      const bool r0 = dl < kp.res_e1, r1 = !r0 && dl < kp.res_e2;
      cnt0 += r0 ? 1u : 0u;
      cnt1 += r1 ? 1u : 0u;
      cnt2 += (!r0 && !r1) ? 1u : 0u;
    }
#pragma unroll
    for (int c = 0; c < C; ++c) xp[c] = x[c];
  }
  if constexpr (WIDE) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q = 0; q < kBins / 2; ++q) {
        acc[c][2 * q] = (uint32_t)acc2[c][q];
        acc[c][2 * q + 1] = (uint32_t)(acc2[c][q] >> 32);
      }
  }
  store_prior<C>(b, p, acc, cnt0, cnt1, cnt2, kp);
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
// The next frame's input is prefetched into registers while the current one
// is processed.  With LP (launches over many frames) the tile's prior records
// are staged into LDS once, so S2 reads no HBM.
template <int C, int K, bool F32, int PPT, bool LP>
__global__ __launch_bounds__(kNT) void k_cascade(Buffers b, Frames fr, KParams kp) {
  constexpr int TILE = kNT * PPT;
  constexpr int R = rec_floats(C, K);
  constexpr int RG = rga_floats(C);
  constexpr int PB = prior_bytes(C);
  __shared__ uint4 s_prior[LP ? TILE * PB / 16 : 1];
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
  if constexpr (LP) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int64_t p = tile0 + j * kNT + tid;
      const int li = j * kNT + tid;
      if (valid[j]) {
        const uint4 *src = reinterpret_cast<const uint4 *>(b.prior + p * PB);
#pragma unroll
        for (int q = 0; q < PB / 16; ++q) s_prior[li * (PB / 16) + q] = src[q];
      }
    }
  }

  // input of the next frame, in flight while the current frame is processed
  float xn[PPT][C];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
#pragma unroll
    for (int c = 0; c < C; ++c) xn[j][c] = 0.0f;
    if (valid[j] && fr.nframes > 0)
      load_px<C, F32>(fr.x, tile0 + j * kNT + tid, xn[j]);
  }

  for (int f = 0; f < fr.nframes; ++f) {
    float x[PPT][C];
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
      for (int c = 0; c < C; ++c) x[j][c] = xn[j][c];
    if (f + 1 < fr.nframes) {
      const void *xf1 = frame_ptr<C, F32>(fr.x, fr.stride, f + 1);
#pragma unroll
      for (int j = 0; j < PPT; ++j)
        if (valid[j]) load_px<C, F32>(xf1, tile0 + j * kNT + tid, xn[j]);
    }
    int st[PPT], pre[PPT];
    bool surv[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int li = j * kNT + tid;
      st[j] = -1;
      surv[j] = false;
      if (valid[j]) {
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
          if (rga_on && dr2 <= kp.lam_r2 * fabsf(rvar[j])) {
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
            const float v = kp.one_m_alpha_rga * fabsf(rvar[j]) + kp.alpha_rga * sr;
            if (!rvar_shared(rvar[j])) rvar[j] = v < kp.var_min ? kp.var_min : v;
            dirty[j] = true;
          } else {
            surv[j] = true;
#pragma unroll
            for (int c = 0; c < C; ++c) s_x[li * C + c] = x[j][c];
            s_dl[li] = dl;
            s_dr2[li] = dr2;
            s_var[li] = fabsf(rvar[j]);
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
        if (fr.partials)
          fr.partials[(int64_t)(f - 1) * fr.nslots + blockIdx.x] =
              stat_row(sp[0], sp[1], sp[2], sp[3], sp[4], sp[5], 0u);
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
          const uint8_t *rec = LP ? reinterpret_cast<const uint8_t *>(&s_prior[li * (PB / 16)])
                                  : b.prior + (tile0 + li) * PB;
          float xl[C];
#pragma unroll
          for (int c = 0; c < C; ++c) xl[c] = s_x[li * C + c];
          conf = confidence<C, F32>(rec, xl, s_dl[li], s_dr2[li], s_var[li], kp);
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
          if (!rvar_shared(rvar[j])) rvar[j] = s_rg[li * (C + 1) + C];
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
    const uint32_t *sp = &s_stat[f & 1][0];
    fr.partials[(int64_t)f * fr.nslots + blockIdx.x] =
        stat_row(sp[0], sp[1], sp[2], sp[3], sp[4], sp[5], 0u);
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
// The fused cascade with one wave per tile of 64*PPT consecutive pixels.
// Same stages as k_cascade, but compaction, the S2/S3 work lists and the
// hand-back of results stay inside one wave: no workgroup barrier, so every
// wave walks its frames independently and the waves of a SIMD overlap each
// other's memory and mixture latencies.
template <int C, int K, bool F32, int PPT, bool LP>
__global__ __launch_bounds__(64) void k_cascade_w(Buffers b, Frames fr, KParams kp) {
  constexpr int TILE = 64 * PPT;
  constexpr int R = rec_floats(C, K);
  constexpr int RG = rga_floats(C);
  constexpr int PB = prior_bytes(C);
  using raw_t = typename RawT<F32>::type;
  __shared__ uint4 s_prior[LP ? TILE * PB / 16 : 1];
  __shared__ float s_x[TILE * C];
  __shared__ float s_dl[TILE];
  __shared__ float s_dr2[TILE];
  __shared__ float s_var[TILE];
  __shared__ float s_conf[TILE];
  __shared__ float s_rg[TILE * (C + 1)];
  __shared__ uint16_t s_la[TILE];
  __shared__ uint16_t s_lb[TILE];
  __shared__ uint8_t s_res[TILE];  // bit0 foreground, bit1 re-seed, bits 2-3 stage

  const int lane = threadIdx.x;
  const int64_t tile0 = (int64_t)blockIdx.x * TILE;
  const bool fd_on = (kp.stage_mask & 1u) != 0;
  const bool rga_on = (kp.stage_mask & 2u) != 0;
  const bool kde_on = (kp.stage_mask & 4u) != 0;

  float xp[PPT][C], rmu[PPT][C], rvar[PPT];
  bool lab[PPT], dirty[PPT], valid[PPT];
  int64_t pc[PPT];  // pixel index clamped into the frame (for the prefetch)
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int64_t p = tile0 + j * 64 + lane;
    valid[j] = p < b.P;
    pc[j] = valid[j] ? p : b.P - 1;
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
      if constexpr (LP) {
        const uint4 *src = reinterpret_cast<const uint4 *>(b.prior + p * PB);
#pragma unroll
        for (int q = 0; q < PB / 16; ++q) s_prior[(j * 64 + lane) * (PB / 16) + q] = src[q];
      }
    }
  }

  // input of the next frame, in flight while the current frame is processed
  raw_t xr[PPT][C];
  uint32_t xw[PPT];
  int npx[PPT];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int64_t rem = b.P - (tile0 + j * 64);
    npx[j] = rem <= 0 ? 0 : (rem >= 64 ? 64 : (int)rem);
    xw[j] = 0u;
#pragma unroll
    for (int c = 0; c < C; ++c) xr[j][c] = 0;
    if (fr.nframes > 0 && npx[j] > 0) {
      if constexpr (F32) raw_load<C, F32>(fr.x, pc[j], xr[j]);
      else xw[j] = u8win_load<C>(static_cast<const uint8_t *>(fr.x), tile0 + j * 64, npx[j], lane);
    }
  }

  for (int f = 0; f < fr.nframes; ++f) {
    float x[PPT][C];
    const void *xf = frame_ptr<C, F32>(fr.x, fr.stride, f);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      if constexpr (F32) raw_to_float<C, F32>(xr[j], x[j]);
      else u8win_extract<C>(xw[j], static_cast<const uint8_t *>(xf), tile0 + j * 64, lane, x[j]);
    }
    {
      // prefetch the next frame (the last frame is re-read: always in bounds)
      const void *xf1 = frame_ptr<C, F32>(fr.x, fr.stride, f + 1 < fr.nframes ? f + 1 : f);
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        if (npx[j] > 0) {
          if constexpr (F32) raw_load<C, F32>(xf1, pc[j], xr[j]);
          else xw[j] = u8win_load<C>(static_cast<const uint8_t *>(xf1), tile0 + j * 64, npx[j], lane);
        }
      }
    }

    // dense: S0 and S1
    int st[PPT];
    bool surv[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int li = j * 64 + lane;
      st[j] = -1;
      surv[j] = false;
      if (valid[j]) {
        const float dl = frame_delta<C>(x[j], xp[j]);
        if (fd_on && dl <= kp.tau_fd) {
          st[j] = 0;
        } else {
          float dr2 = 0.0f;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const float d = x[j][c] - rmu[j][c];
            dr2 = dr2 + d * d;
          }
          if (rga_on && dr2 <= kp.lam_r2 * fabsf(rvar[j])) {
            st[j] = 1;
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
            const float v = kp.one_m_alpha_rga * fabsf(rvar[j]) + kp.alpha_rga * sr;
            if (!rvar_shared(rvar[j])) rvar[j] = v < kp.var_min ? kp.var_min : v;
            dirty[j] = true;
          } else {
            surv[j] = true;
#pragma unroll
            for (int c = 0; c < C; ++c) s_x[li * C + c] = x[j][c];
            s_dl[li] = dl;
            s_dr2[li] = dr2;
            s_var[li] = fabsf(rvar[j]);
          }
        }
      }
    }
    // list A: S1 survivors in pixel order
    int nA = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const unsigned long long bal = __ballot(surv[j]);
      if (surv[j]) s_la[nA + lane_prefix(bal)] = (uint16_t)(j * 64 + lane);
      nA += (int)__popcll(bal);
    }
    wave_sync();

    // S2 over list A, survivors into list B
    int nB = 0;
    for (int r0 = 0; r0 < nA; r0 += 64) {
      const int i = r0 + lane;
      bool go3 = false;
      int li = 0;
      if (i < nA) {
        li = s_la[i];
        float conf = 0.0f;
        bool accept = false;
        if (kde_on) {
          const uint8_t *rec = LP ? reinterpret_cast<const uint8_t *>(&s_prior[li * (PB / 16)])
                                  : b.prior + (tile0 + li) * PB;
          float xl[C];
#pragma unroll
          for (int c = 0; c < C; ++c) xl[c] = s_x[li * C + c];
          conf = confidence<C, F32>(rec, xl, s_dl[li], s_dr2[li], s_var[li], kp);
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
      if (go3) s_lb[nB + lane_prefix(bal)] = (uint16_t)li;
      nB += (int)__popcll(bal);
    }
    wave_sync();

    // S3 over list B
    for (int i = lane; i < nB; i += 64) {
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
    wave_sync();

    // hand-back, mask, level statistics
    uint8_t *mk = fr.mask ? fr.mask + (int64_t)f * fr.mstride : nullptr;
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c3bg = 0, cfg = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int li = j * 64 + lane;
      if (surv[j]) {
        const uint8_t r = s_res[li];
        lab[j] = (r & 1) != 0;
        st[j] = r >> 2;
        if (r & 2) {
#pragma unroll
          for (int c = 0; c < C; ++c) rmu[j][c] = s_rg[li * (C + 1) + c];
          if (!rvar_shared(rvar[j])) rvar[j] = s_rg[li * (C + 1) + C];
          dirty[j] = true;
        }
      }
      if (valid[j]) {
        if (mk) mk[tile0 + li] = lab[j] ? 255 : 0;
#pragma unroll
        for (int c = 0; c < C; ++c) xp[j][c] = x[j][c];
      }
      if (fr.partials) {
        c0 += (uint32_t)__popcll(__ballot(st[j] == 0));
        c1 += (uint32_t)__popcll(__ballot(st[j] == 1));
        c2 += (uint32_t)__popcll(__ballot(st[j] == 2));
        c3 += (uint32_t)__popcll(__ballot(st[j] == 3));
        c3bg += (uint32_t)__popcll(__ballot(st[j] == 3 && !lab[j]));
        cfg += (uint32_t)__popcll(__ballot(valid[j] && lab[j]));
      }
    }
    if (fr.partials && lane == 0)
      fr.partials[(int64_t)f * fr.nslots + blockIdx.x] = stat_row(c0, c1, c2, c3, c3bg, cfg, 0u);
    wave_sync();
  }

#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int64_t p = tile0 + j * 64 + lane;
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
    if (lane == 0 && tile0 + j * 64 < b.P) b.labels[(tile0 + j * 64) >> 6] = bal;
  }
}


// ============================================================================
// The cascade with one wave per 64 consecutive pixels and one pixel per lane.
// A wave never holds more than 64 survivors, so S2 and S3 take one pass
// whether or not the survivors are compacted; here each survivor stays in its
// own lane, which keeps list hand-offs off the per-frame critical path.
// (The compacting kernels above pool the survivors of 128..1024 pixels into
// dense lists instead.)
//  - dense state (previous value, label, running average) in registers for
//    the whole launch;
//  - a pixel's mixture record is read from HBM when the launch starts (launches
//    of kEagerRecordFrames frames or more) or the first time the pixel
//    reaches S3 (the load is issued before S2 runs), and then stays in
//    registers -- only this lane ever touches it -- and is written back once
//    at the end of the launch;
//  - the input is block-staged through LDS (InStage): the global-memory wait
//    is paid once per block of frames, on loads issued a block earlier;
//  - frames go two per loop iteration, the input alternating between two
//    register arrays, so the previous value is never copied;
//  - the mask and statistics stores are bounds-checked buffer stores;
//  - for u8 input up to K = 5 the register budget keeps five waves per SIMD (a 640x480
//    frame is 4.7 waves per SIMD: all of them stay resident).
// Launches of at least this many frames load every pixel's mixture record at
// their start (shorter ones when the pixel first reaches S3).
constexpr int kEagerRecordFrames = 32;

// LDS of one wave running cascade_tile: the tile's prior records (when
// staged) and the input ring.
template <int C, bool F32, bool LP>
struct TileLds {
  static constexpr int NB = 8;  // frames per input block
  uint4 prior[LP ? 64 * prior_bytes(C) / 16 : 1];
  uint32_t in[NB * InStage<C, F32, NB>::NDW * 64];
};

// The cascade over fr.nframes frames for the 64 pixels of one tile (tile =
// index of the 64-pixel run within the stream), one pixel per lane.  Shared
// by the one-stream kernel and the batched tick.
template <int C, int K, bool F32, bool LP, bool SAMP>
__device__ __forceinline__ void cascade_tile(const Buffers &b, const Frames &fr, const KParams &kp,
                                             int64_t tile, int lane, TileLds<C, F32, LP> &lds) {
  constexpr int R = rec_floats(C, K);
  constexpr int RG = rga_floats(C);
  constexpr int PB = prior_bytes(C);
  constexpr int NB = TileLds<C, F32, LP>::NB;
  using Stage = InStage<C, F32, NB>;
  uint4 *s_prior = lds.prior;
  uint32_t *s_in = lds.in;

  const int64_t tile0 = tile * 64;
  const int64_t p = tile0 + lane;
  const bool valid = p < b.P;
  const int64_t pcl = valid ? p : b.P - 1;
  const int64_t rem = b.P - tile0;
  const int npx = rem >= 64 ? 64 : (int)rem;
  const bool fd_on = (kp.stage_mask & 1u) != 0;
  const bool rga_on = (kp.stage_mask & 2u) != 0;
  const bool kde_on = (kp.stage_mask & 4u) != 0;
  const bool tau_zero = kp.tau_fd == 0.0f;

  float xp[C], rmu[C], rvar = 0.0f;
  // per-lane flags kept as integers (0/1) so that branch joins cost no
  // lane-mask bookkeeping
  uint32_t lab = 0u, dirty = 0u, have_rec = 0u, rec_dirty = 0u;
#pragma unroll
  for (int c = 0; c < C; ++c) xp[c] = rmu[c] = 0.0f;
  if (valid) {
    lab = (uint32_t)((b.labels[p >> 6] >> lane) & 1ull);
    load_px<C, F32>(b.prev, p, xp);
    const float *rg = b.rga + p * RG;
#pragma unroll
    for (int c = 0; c < C; ++c) rmu[c] = rg[c];
    rvar = rg[C];
    if constexpr (LP) {
      const uint4 *src = reinterpret_cast<const uint4 *>(b.prior + p * PB);
#pragma unroll
      for (int q = 0; q < PB / 16; ++q) s_prior[lane * (PB / 16) + q] = src[q];
    }
  }
  // sampling (§2 "Confidence based temporal sampling"): the lane's count of
  // consecutive confident frames (lanes past the end count as saturated) and
  // the block's phase (frame + block) % period for frame 0
  uint32_t sat = 0xffffu, ph = 0u;
  if constexpr (SAMP) {
    if (valid) sat = b.sat[p];
    ph = (uint32_t)((fr.frame0 + tile) % (int64_t)kp.samp_period);
  }
  // a lane reads back only its own staged record, so no wave-level sync is needed
  const uint8_t *prec = LP ? reinterpret_cast<const uint8_t *>(&s_prior[lane * (PB / 16)])
                           : b.prior + pcl * PB;
  float *grec = b.gmm + pcl * R;
  Mix<C, K> m;  // the pixel's mixture, valid once have_rec
  // A long launch requests every record at its start: most pixels reach S3
  // at some frame of a long run, and a record first requested inside the
  // frame loop stalls the whole wave on one memory round trip.
  if (fr.nframes >= kEagerRecordFrames) {
    if (valid) rec_load<C, K>(grec, m);
    have_rec = 1u;
  }

  // byte offset of the lane's pixel in a frame's mask, and of the lane's
  // statistics word in a frame's row; out-of-range lanes are dropped by the
  // buffer stores' bounds check
  const int moff = valid ? (int)p : 0x7fffffff;
  const int soff = lane == 0 ? (int)(tile * 16) : 0x7fffffff;
  const int srow = fr.nslots * 16;  // bytes per frame of statistics rows

  // misalignment of the tile's input run within 4 bytes, frame by frame
  const int in_bytes = F32 ? 4 : 1;
  const int mis0 = (int)((reinterpret_cast<uintptr_t>(fr.x) + (uint64_t)tile0 * C * in_bytes) & 3);
  const int mis_step = (int)(((uint64_t)fr.stride * in_bytes) & 3);

  Stage in;
  if (fr.nframes > 0) in.issue(fr.x, fr.stride, fr.nframes, 0, tile0, npx, lane);

  for (int f0 = 0; f0 < fr.nframes; f0 += NB) {
    in.commit(s_in, lane);
    wave_sync();
    in.issue(fr.x, fr.stride, fr.nframes, f0 + NB, tile0, npx, lane);
    const int nk = fr.nframes - f0 < NB ? fr.nframes - f0 : NB;
    // this block's masks and statistics rows (frame k at soffset k * row);
    // the record count is an unsigned 32-bit field: at most 8 * 2^28 = 2^31
    // mask bytes (frames are limited to 2^28 pixels)
    const __amdgpu_buffer_rsrc_t mr = __builtin_amdgcn_make_buffer_rsrc(
        fr.mask ? fr.mask + (int64_t)f0 * fr.mstride : nullptr, (short)0,
        fr.mask ? (int)(uint32_t)((uint64_t)nk * (uint64_t)fr.mstride) : 0, 0x00020000);
    const __amdgpu_buffer_rsrc_t sr = __builtin_amdgcn_make_buffer_rsrc(
        fr.partials ? fr.partials + (int64_t)f0 * fr.nslots : nullptr, (short)0,
        fr.partials ? nk * srow : 0, 0x00020000);
    int mis = (mis0 + f0 * mis_step) & 3;

    // one frame: reads the input into x; xq holds the previous frame's value.
    // Frames alternate between two arrays, so no copy of x into the previous
    // value is needed.
    auto frame = [&](int k, int mis, float (&x)[C], const float (&xq)[C]) {
        bool halted = false;
        if constexpr (SAMP) {
          // a block whose pixels are all saturated is evaluated only in phase;
          // when halted the labels repeat, no level runs and nothing adapts
          halted = ph != 0u && __ballot(sat < kp.samp_window) == 0ull;
          ph = ph + 1u == kp.samp_period ? 0u : ph + 1u;
        }
        // this frame's level, as lane flags read only by the statistics
        // (S0, S1, S2 accepts, survivors of S2; halted lanes set none)
        bool e0 = false, e1 = false, e2 = false, e3 = false;
        if (!halted) {
          Stage::read_mis(s_in, k, mis, lane, x);

          // S0 (frame difference) and S1 (running average) for every lane;
          // with u8 input and a zero tolerance S0 is plain equality, and the
          // difference itself is formed only for survivors
          bool fd_ok;
          if (!F32 && tau_zero) {
            fd_ok = true;
#pragma unroll
            for (int c = 0; c < C; ++c) fd_ok = fd_ok && x[c] == xq[c];
          } else {
            float d0 = 0.0f;
#pragma unroll
            for (int c = 0; c < C; ++c) d0 = fmaxf(d0, fabsf(x[c] - xq[c]));
            fd_ok = d0 <= kp.tau_fd;
          }
          float dr2 = 0.0f;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            const float d = x[c] - rmu[c];
            dr2 = dr2 + d * d;
          }
          const bool s0 = fd_on && fd_ok;
          const bool s1 = !s0 && rga_on && dr2 <= kp.lam_r2 * fabsf(rvar);
          if constexpr (SAMP) {
            // confident: decided by the frame difference, or by the running
            // average within samp_lambda standard deviations (its variance before
            // this frame's update)
            const bool conf = s0 || (s1 && dr2 <= kp.lam_s2 * fabsf(rvar));
            const uint32_t nsat = conf ? (sat < 65535u ? sat + 1u : 65535u) : 0u;
            sat = valid ? nsat : sat;
          }
          {
            float nmu[C];
#pragma unroll
            for (int c = 0; c < C; ++c) nmu[c] = kp.one_m_alpha_rga * rmu[c] + kp.alpha_rga * x[c];
            float sr = 0.0f;
#pragma unroll
            for (int c = 0; c < C; ++c) {
              const float e = x[c] - nmu[c];
              sr = sr + e * e;
            }
            const float nv = kp.one_m_alpha_rga * fabsf(rvar) + kp.alpha_rga * sr;
            // u8 input keeps both operands positive and finite, where the
            // larger binary32 is the larger bit pattern
            const float nvar = F32 ? fmaxf(kp.var_min, nv)
                                   : __int_as_float(max(__float_as_int(kp.var_min), __float_as_int(nv)));
#pragma unroll
            for (int c = 0; c < C; ++c) rmu[c] = s1 ? nmu[c] : rmu[c];
            rvar = s1 && !rvar_shared(rvar) ? nvar : rvar;
          }
          dirty |= s1 ? 1u : 0u;
          lab = s1 ? 0u : lab;
          e0 = valid && s0;
          e1 = valid && s1;

          if (valid && !s0 && !s1) {
            // survivor: first time in this launch, the mixture record is
            // requested before S2 runs
            if (!have_rec) {
              rec_load<C, K>(grec, m);
              have_rec = 1u;
            }
            float conf = 0.0f;
            bool accept = false;
            if (kde_on) {
              float dl = 0.0f;
#pragma unroll
              for (int c = 0; c < C; ++c) dl = fmaxf(dl, fabsf(x[c] - xq[c]));
              conf = confidence<C, F32>(prec, x, dl, dr2, fabsf(rvar), kp);
              accept = conf >= kp.conf_thr;
            }
            if (accept) {
              e2 = true;  // S2: background by the scene prior, nothing adapts
              lab = 0u;
            } else {
              // S3: the full mixture with the confidence-driven rate
              e3 = true;
              const float ae = kp.alpha * (1.0f - kp.kappa * conf);
              int l, mp;
              mix_step<C, K>(m, x, ae, kp, l, mp);
              rec_dirty = 1u;
              lab = l ? 1u : 0u;
              if (!l) {
                // background from the mixture: the running average takes the
                // matched component (the transition update of the active level)
                float sv = m.var[0];
#pragma unroll
                for (int c = 0; c < C; ++c) rmu[c] = m.mu[0][c];
#pragma unroll
                for (int kk = 1; kk < K; ++kk) {
                  if (mp == kk) {
                    sv = m.var[kk];
#pragma unroll
                    for (int c = 0; c < C; ++c) rmu[c] = m.mu[kk][c];
                  }
                }
                rvar = rvar_shared(rvar) ? rvar : sv;
                dirty = 1u;
              }
            }
          }
        } else {
#pragma unroll
          for (int c = 0; c < C; ++c) x[c] = xq[c];
        }
        // masks are streamed out: non-temporal (cache policy bit 1)
        __builtin_amdgcn_raw_buffer_store_b8((unsigned char)(lab ? 255 : 0), mr, moff,
                                             k * (int)fr.mstride, 2);
        if (fr.partials) {
          const uint32_t c0 = (uint32_t)__popcll(__ballot(e0));
          const uint32_t c1 = (uint32_t)__popcll(__ballot(e1));
          const uint32_t c2 = (uint32_t)__popcll(__ballot(e2));
          const uint32_t c3 = (uint32_t)__popcll(__ballot(e3));
          const uint32_t c3bg = (uint32_t)__popcll(__ballot(e3 && !lab));
          const uint32_t cfg = (uint32_t)__popcll(__ballot(valid && lab));
          const uint32_t csk = SAMP ? (uint32_t)__popcll(__ballot(halted && valid)) : 0u;
          const uint4 row = stat_row(c0, c1, c2, c3, c3bg, cfg, csk);
          typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));
          const v4u32 rv = {row.x, row.y, row.z, row.w};
          __builtin_amdgcn_raw_buffer_store_b128(rv, sr, soff, k * srow, 0);
        }
    };
    for (int k = 0; k < nk; k += 2) {
      float xb[C];
      frame(k, mis, xb, xp);
      mis = (mis + mis_step) & 3;
      if (k + 1 < nk) {
        frame(k + 1, mis, xp, xb);
        mis = (mis + mis_step) & 3;
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) xp[c] = xb[c];
      }
    }
    wave_sync();
  }

  if (valid) {
    if (rec_dirty) rec_store<C, K>(grec, m);
    if (dirty) {
      float *rg = b.rga + p * RG;
#pragma unroll
      for (int c = 0; c < C; ++c) rg[c] = rmu[c];
      rg[C] = rvar;
    }
    store_px<C, F32>(b.prev, p, xp);
    if constexpr (SAMP) b.sat[p] = (uint16_t)sat;
  }
  const unsigned long long bal = __ballot(valid && lab);
  if (lane == 0) b.labels[tile0 >> 6] = bal;
}

// Waves per SIMD the one-wave cascade kernels are held to: five for u8 input
// up to K=5 (at most 96 VGPRs, every wave of a 640x480 frame resident; with
// frames handled in pairs the kernels need 76, the sampling variant 78).
__host__ __device__ constexpr int cascade_min_waves(bool f32, int K, bool samp) {
  (void)samp;
  return (!f32 && K <= 5) ? 5 : 1;
}

template <int C, int K, bool F32, bool LP, bool SAMP>
__global__ __launch_bounds__(64, cascade_min_waves(F32, K, SAMP)) void k_cascade_d(Buffers b, Frames fr, KParams kp) {
  __shared__ TileLds<C, F32, LP> lds;
  // Tiles follow the workgroup order, which the dispatcher deals round-robin
  // over the XCDs: the spatially clustered survivor work (foreground, bimodal
  // regions) is spread evenly over the chip.  (Contiguous tile runs per XCD
  // share boundary cache lines but concentrate that work; measured slower.)
  cascade_tile<C, K, F32, LP, SAMP>(b, fr, kp, blockIdx.x, threadIdx.x, lds);
}

// ============================================================================
// The cascade for one frame per launch (a live camera's cog_step), where the
// dense state streams from HBM every frame.  One wave per 256 consecutive
// pixels; lane l owns pixels 4l .. 4l+3 of the tile, so a lane's input,
// previous value, running average and mask are contiguous and move in wide
// loads and stores.  S0 and S1 run for every pixel in the owning lane; the
// tile's S1 survivors are compacted into a wave-level LDS work list (ballot,
// mbcnt prefix) with what S2 needs, and S2/S3 run over the list one survivor
// per lane: a pass carries up to 64 survivors of 256 pixels, where
// one-pixel-per-lane tiles leave most lanes of an S3 pass idle.  The results
// go back to the owners through LDS for the mask, label and statistics.
// Pixel arithmetic and order are those of cascade_tile, so the two agree bit
// for bit.
constexpr int kFramePx = kFrameTile / 64;  // pixels per lane

template <int C, bool F32>
struct FrameLds {
  static constexpr int NXW = F32 ? C : 1;
  uint16_t li[kFrameTile];           // work list: pixel within the tile
  uint32_t xw[NXW][kFrameTile];      // the survivor's input (u8: packed bytes)
  float dl[kFrameTile], dr2[kFrameTile], var[kFrameTile];
  uint8_t res[kFrameTile];           // per pixel: bit 0 label, bit 1 S2 accept, bit 2 S3
};

// Bits 4j .. 4j+3 of a 16-bit value spread to every fourth bit (bit k to 4k).
__device__ __forceinline__ uint64_t spread4(uint64_t v) {
  v &= 0xffffull;
  v = (v | (v << 24)) & 0x000000ff000000ffull;
  v = (v | (v << 12)) & 0x000f000f000f000full;
  v = (v | (v << 6)) & 0x0303030303030303ull;
  v = (v | (v << 3)) & 0x1111111111111111ull;
  return v;
}

template <int C, int K, bool F32>
__device__ __forceinline__ void frame_tile(const Buffers &b, const Frames &fr, const KParams &kp,
                                           int64_t tile, int lane, FrameLds<C, F32> &lds) {
  constexpr int PX = kFramePx;
  constexpr int R = rec_floats(C, K);
  constexpr int RG = rga_floats(C);
  constexpr int PB = prior_bytes(C);
  // input dwords of a lane's PX pixels (u8: PX*C bytes; f32: PX*C floats)
  constexpr int NDW = F32 ? PX * C : (PX * C) / 4;
  static_assert(F32 || (PX * C) % 4 == 0, "u8 lanes hold whole dwords");

  const int64_t tile0 = tile * kFrameTile;
  const int64_t p0 = tile0 + PX * lane;
  const bool fd_on = (kp.stage_mask & 1u) != 0;
  const bool rga_on = (kp.stage_mask & 2u) != 0;
  const bool kde_on = (kp.stage_mask & 4u) != 0;
  const bool tau_zero = kp.tau_fd == 0.0f;
  // wide path: the whole tile exists and the caller's frame and mask are
  // dword-aligned (state arrays are 256-byte aligned)
  const bool wide = tile0 + kFrameTile <= b.P &&
                    ((reinterpret_cast<uintptr_t>(fr.x) | reinterpret_cast<uintptr_t>(fr.mask)) & 3) == 0;

  bool valid[PX];
  float x[PX][C], xp[PX][C], rmu[PX][C], rvar[PX];
  uint32_t raw[NDW];
  uint32_t lab4 = 0u;  // the lane's PX label bits (one word holds the labels of 16 lanes)
#pragma unroll
  for (int j = 0; j < PX; ++j) valid[j] = p0 + j < b.P;
  if (wide) {
    // every load of the dense levels issued at once: one memory round trip
    const uint32_t *qx = reinterpret_cast<const uint32_t *>(
        static_cast<const char *>(fr.x) + p0 * C * (F32 ? 4 : 1));
    const uint32_t *qp = reinterpret_cast<const uint32_t *>(
        static_cast<const char *>(b.prev) + p0 * C * (F32 ? 4 : 1));
    uint32_t rp[NDW];
    float rgv[PX][RG];
#pragma unroll
    for (int d = 0; d < NDW; ++d) raw[d] = __builtin_nontemporal_load(qx + d);
#pragma unroll
    for (int d = 0; d < NDW; ++d) rp[d] = qp[d];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
      const float *rg = b.rga + (p0 + j) * RG;
      if constexpr (RG == 4) {
        const float4 v = *reinterpret_cast<const float4 *>(rg);
        rgv[j][0] = v.x;
        rgv[j][1] = v.y;
        rgv[j][2] = v.z;
        rgv[j][3] = v.w;
      } else {
        const float2 v = *reinterpret_cast<const float2 *>(rg);
        rgv[j][0] = v.x;
        rgv[j][1] = v.y;
      }
    }
    const unsigned long long lw = b.labels[p0 >> 6];
#pragma unroll
    for (int j = 0; j < PX; ++j) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int e = j * C + c;
        if constexpr (F32) {
          x[j][c] = __uint_as_float(raw[e]);
          xp[j][c] = __uint_as_float(rp[e]);
        } else {
          x[j][c] = (float)((raw[e >> 2] >> (8 * (e & 3))) & 0xffu);
          xp[j][c] = (float)((rp[e >> 2] >> (8 * (e & 3))) & 0xffu);
        }
        rmu[j][c] = rgv[j][c];
      }
      rvar[j] = rgv[j][RG - 1];
    }
    lab4 = (uint32_t)((lw >> (p0 & 63)) & 0xfull);
  } else {
#pragma unroll
    for (int d = 0; d < NDW; ++d) raw[d] = 0u;
#pragma unroll
    for (int j = 0; j < PX; ++j) {
      rvar[j] = 0.0f;
#pragma unroll
      for (int c = 0; c < C; ++c) x[j][c] = xp[j][c] = rmu[j][c] = 0.0f;
      if (valid[j]) {
        load_px<C, F32>(fr.x, p0 + j, x[j]);
        load_px<C, F32>(b.prev, p0 + j, xp[j]);
        const float *rg = b.rga + (p0 + j) * RG;
#pragma unroll
        for (int c = 0; c < C; ++c) rmu[j][c] = rg[c];
        rvar[j] = rg[RG - 1];
      }
    }
    if (p0 < b.P) lab4 = (uint32_t)((b.labels[p0 >> 6] >> (p0 & 63)) & 0xfull);
  }

  // ---- dense levels: S0 (frame difference) and S1 (running average)
  bool s0[PX], s1[PX], surv[PX];
  float dr2[PX];
#pragma unroll
  for (int j = 0; j < PX; ++j) {
    bool fd_ok;
    if (!F32 && tau_zero) {
      fd_ok = true;
#pragma unroll
      for (int c = 0; c < C; ++c) fd_ok = fd_ok && x[j][c] == xp[j][c];
    } else {
      float d0 = 0.0f;
#pragma unroll
      for (int c = 0; c < C; ++c) d0 = fmaxf(d0, fabsf(x[j][c] - xp[j][c]));
      fd_ok = d0 <= kp.tau_fd;
    }
    float d2 = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const float d = x[j][c] - rmu[j][c];
      d2 = d2 + d * d;
    }
    dr2[j] = d2;
    s0[j] = valid[j] && fd_on && fd_ok;
    s1[j] = valid[j] && !s0[j] && rga_on && d2 <= kp.lam_r2 * fabsf(rvar[j]);
    surv[j] = valid[j] && !s0[j] && !s1[j];
    if (s1[j]) lab4 &= ~(1u << j);
  }

  // ---- the owner's writes that do not depend on S2/S3: previous value, and
  // the running average of every S1 accept (EMA of mean and variance)
  if (wide) {
    uint32_t *qp = reinterpret_cast<uint32_t *>(static_cast<char *>(b.prev) + p0 * C * (F32 ? 4 : 1));
#pragma unroll
    for (int d = 0; d < NDW; ++d) qp[d] = raw[d];
  } else {
#pragma unroll
    for (int j = 0; j < PX; ++j)
      if (valid[j]) store_px<C, F32>(b.prev, p0 + j, x[j]);
  }
#pragma unroll
  for (int j = 0; j < PX; ++j) {
    if (s1[j]) {
      float nmu[C];
#pragma unroll
      for (int c = 0; c < C; ++c) nmu[c] = kp.one_m_alpha_rga * rmu[j][c] + kp.alpha_rga * x[j][c];
      float sr = 0.0f;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const float e = x[j][c] - nmu[c];
        sr = sr + e * e;
      }
      const float nv = kp.one_m_alpha_rga * fabsf(rvar[j]) + kp.alpha_rga * sr;
      float nvar = F32 ? fmaxf(kp.var_min, nv)
                       : __int_as_float(max(__float_as_int(kp.var_min), __float_as_int(nv)));
      nvar = rvar_shared(rvar[j]) ? rvar[j] : nvar;
      float *rg = b.rga + (p0 + j) * RG;
      if constexpr (RG == 4) *reinterpret_cast<float4 *>(rg) = make_float4(nmu[0], nmu[1], nmu[2], nvar);
      else *reinterpret_cast<float2 *>(rg) = make_float2(nmu[0], nvar);
    }
  }

  // ---- work list of the S1 survivors
  int nA = 0;
#pragma unroll
  for (int j = 0; j < PX; ++j) {
    const unsigned long long bal = __ballot(surv[j]);
    if (surv[j]) {
      const int pos = nA + lane_prefix(bal);
      lds.li[pos] = (uint16_t)(PX * lane + j);
      if constexpr (F32) {
#pragma unroll
        for (int c = 0; c < C; ++c) lds.xw[c][pos] = __float_as_uint(x[j][c]);
      } else {
        uint32_t w = 0u;
#pragma unroll
        for (int c = 0; c < C; ++c) w |= (uint32_t)x[j][c] << (8 * c);
        lds.xw[0][pos] = w;
      }
      float dl = 0.0f;
#pragma unroll
      for (int c = 0; c < C; ++c) dl = fmaxf(dl, fabsf(x[j][c] - xp[j][c]));
      lds.dl[pos] = dl;
      lds.dr2[pos] = dr2[j];
      lds.var[pos] = rvar[j];
    }
    nA += (int)__popcll(bal);
  }
  wave_sync();

  // ---- S2 and S3 over the list, one survivor per lane
  for (int r0 = 0; r0 < nA; r0 += 64) {
    const int i = r0 + lane;
    if (i < nA) {
      const int li = lds.li[i];
      const int64_t p = tile0 + li;
      float xs[C];
      if constexpr (F32) {
#pragma unroll
        for (int c = 0; c < C; ++c) xs[c] = __uint_as_float(lds.xw[c][i]);
      } else {
        const uint32_t w = lds.xw[0][i];
#pragma unroll
        for (int c = 0; c < C; ++c) xs[c] = (float)((w >> (8 * c)) & 0xffu);
      }
      float *grec = b.gmm + p * R;
      Mix<C, K> m;
      rec_load<C, K>(grec, m);  // requested before S2 runs
      float conf = 0.0f;
      bool accept = false;
      if (kde_on) {
        conf = confidence<C, F32>(b.prior + p * PB, xs, lds.dl[i], lds.dr2[i], fabsf(lds.var[i]),
                                  kp);
        accept = conf >= kp.conf_thr;
      }
      uint32_t res;
      if (accept) {
        res = 2u;  // S2: background by the scene prior, nothing adapts
      } else {
        const float ae = kp.alpha * (1.0f - kp.kappa * conf);
        int l, mp;
        mix_step<C, K>(m, xs, ae, kp, l, mp);
        rec_store<C, K>(grec, m);
        res = 4u | (l ? 1u : 0u);
        if (!l) {
          // background from the mixture: the running average takes the
          // matched component
          float sm[C], sv = m.var[0];
#pragma unroll
          for (int c = 0; c < C; ++c) sm[c] = m.mu[0][c];
#pragma unroll
          for (int kk = 1; kk < K; ++kk) {
            if (mp == kk) {
              sv = m.var[kk];
#pragma unroll
              for (int c = 0; c < C; ++c) sm[c] = m.mu[kk][c];
            }
          }
          sv = rvar_shared(lds.var[i]) ? lds.var[i] : sv;
          float *rg = b.rga + p * RG;
          if constexpr (RG == 4) *reinterpret_cast<float4 *>(rg) = make_float4(sm[0], sm[1], sm[2], sv);
          else *reinterpret_cast<float2 *>(rg) = make_float2(sm[0], sv);
        }
      }
      lds.res[li] = (uint8_t)res;
    }
  }
  wave_sync();

  // ---- results back to the owners: mask, labels, level statistics
  bool e2[PX], e3[PX];
#pragma unroll
  for (int j = 0; j < PX; ++j) {
    e2[j] = e3[j] = false;
    if (surv[j]) {
      const uint32_t r = lds.res[PX * lane + j];
      e2[j] = (r & 2u) != 0;
      e3[j] = (r & 4u) != 0;
      lab4 = (r & 1u) ? (lab4 | (1u << j)) : (lab4 & ~(1u << j));
    }
  }
  if (fr.mask) {
    if (wide) {
      uint32_t mw = 0u;
#pragma unroll
      for (int j = 0; j < PX; ++j) mw |= ((lab4 >> j) & 1u) ? (0xffu << (8 * j)) : 0u;
      __builtin_nontemporal_store(mw, reinterpret_cast<uint32_t *>(fr.mask + p0));
    } else {
#pragma unroll
      for (int j = 0; j < PX; ++j)
        if (valid[j]) fr.mask[p0 + j] = ((lab4 >> j) & 1u) ? 255 : 0;
    }
  }
  // label words: word q holds lanes 16q .. 16q+15, four bits each
  unsigned long long bal[PX];
#pragma unroll
  for (int j = 0; j < PX; ++j) bal[j] = __ballot(valid[j] && ((lab4 >> j) & 1u));
  if (lane < PX && tile0 + 64 * lane < b.P) {
    const int sh = 16 * lane;
    uint64_t word = 0ull;
#pragma unroll
    for (int j = 0; j < PX; ++j) word |= spread4(bal[j] >> sh) << j;
    b.labels[(tile0 >> 6) + lane] = word;
  }
  if (fr.partials) {
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c3bg = 0, cfg = 0;
#pragma unroll
    for (int j = 0; j < PX; ++j) {
      c0 += (uint32_t)__popcll(__ballot(s0[j]));
      c1 += (uint32_t)__popcll(__ballot(s1[j]));
      c2 += (uint32_t)__popcll(__ballot(e2[j]));
      c3 += (uint32_t)__popcll(__ballot(e3[j]));
      c3bg += (uint32_t)__popcll(__ballot(e3[j] && !((lab4 >> j) & 1u)));
      cfg += (uint32_t)__popcll(bal[j]);
    }
    if (lane == 0) fr.partials[tile] = stat_row(c0, c1, c2, c3, c3bg, cfg, 0u);
  }
}

template <int C, int K, bool F32>
__global__ __launch_bounds__(64) void k_frame(Buffers b, Frames fr, KParams kp) {
  __shared__ FrameLds<C, F32> lds;
  frame_tile<C, K, F32>(b, fr, kp, blockIdx.x, threadIdx.x, lds);
}

// ============================================================================
// Batched tick: many streams of one class in one persistent launch.  The
// tick's tiles (64 pixels each) are numbered over its items; a schedule unit
// is `group` consecutive tiles.  Units go round-robin over the workgroups
// (static) or are taken from an atomic counter (dynamic); either way a
// wave's units increase, so its item cursor only moves forward.  Item and
// slot descriptors are read through the constant address space, so they
// arrive in scalar registers.
typedef const __attribute__((address_space(4))) TickItem CTickItem;
typedef const __attribute__((address_space(4))) TickHead CTickHead;

// A descriptor field copied out through the constant address space, word by
// word (the copy constructors do not take address-space-4 references).
template <typename T>
__device__ __forceinline__ T const_copy(const T *src) {
  static_assert(sizeof(T) % 4 == 0, "descriptor fields are whole words");
  typedef const __attribute__((address_space(4))) uint32_t CWord;
  CWord *w = (CWord *)src;
  T v;
  uint32_t *d = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = w[i];
  return v;
}

__device__ __forceinline__ int take_unit(uint32_t *queue, int lane) {
  uint32_t v = 0u;
  if (lane == 0) v = atomicAdd(queue, 1u);
  return (int)__builtin_amdgcn_readfirstlane(v);
}

// Tile and unit indices are 32-bit: the host keeps a tick below 2^31 tiles.
template <int C, int K, bool F32, bool LP, bool SAMP>
__global__ __launch_bounds__(64, cascade_min_waves(F32, K, SAMP)) void k_tick(TickHead *head,
                                                                      const TickItem *items,
                                                                      int dynamic) {
  __shared__ TileLds<C, F32, LP> lds;
  const int lane = threadIdx.x;
  CTickHead *ch = (CTickHead *)head;
  CTickItem *ci = (CTickItem *)items;
  const int total = (int)ch->total_tiles;
  const int group = ch->group;
  const int units = (total + group - 1) / group;
  uint32_t *queue = &head->queue;
  int u = dynamic ? take_unit(queue, lane) : (int)blockIdx.x;
  int it = 0;
  while (u < units) {
    // the next unit is requested before this one runs
    const int nxt = dynamic ? take_unit(queue, lane) : u + (int)gridDim.x;
    const int t1 = u < units - 1 ? (u + 1) * group : total;
    for (int t = u * group; t < t1; ++t) {
      while (it + 1 < ch->n_items && (int)ci[it + 1].tile_begin <= t) ++it;
      const Frames fr = const_copy(&items[it].fr);
      const Buffers b = const_copy(&items[it].b);
      const KParams kp = const_copy(&items[it].kp);
      cascade_tile<C, K, F32, LP, SAMP>(b, fr, kp, t - (int)ci[it].tile_begin, lane, lds);
    }
    u = nxt;
  }
}

// The batched tick's compacting variant: every item of the launch advances by
// exactly one frame (no sampling), in the per-frame kernel's 256-pixel tiles
// (frame_tile), numbered over the items as in k_tick.
template <int C, int K, bool F32>
__global__ __launch_bounds__(64) void k_tick_c(TickHead *head, const TickItem *items, int dynamic) {
  __shared__ FrameLds<C, F32> lds;
  const int lane = threadIdx.x;
  CTickHead *ch = (CTickHead *)head;
  CTickItem *ci = (CTickItem *)items;
  const int total = (int)ch->total_tiles;
  const int group = ch->group;
  const int units = (total + group - 1) / group;
  uint32_t *queue = &head->queue;
  int u = dynamic ? take_unit(queue, lane) : (int)blockIdx.x;
  int it = 0;
  while (u < units) {
    const int nxt = dynamic ? take_unit(queue, lane) : u + (int)gridDim.x;
    const int t1 = u < units - 1 ? (u + 1) * group : total;
    for (int t = u * group; t < t1; ++t) {
      while (it + 1 < ch->n_items && (int)ci[it + 1].tile_begin <= t) ++it;
      const Frames fr = const_copy(&items[it].fr);
      const Buffers b = const_copy(&items[it].b);
      const KParams kp = const_copy(&items[it].kp);
      frame_tile<C, K, F32>(b, fr, kp, t - (int)ci[it].tile_begin, lane, lds);
      wave_sync();  // the next tile reuses the work list
    }
    u = nxt;
  }
}

// ============================================================================
// Plain Stauffer-Grimson baseline: every pixel runs the mixture step every
// frame (alpha fixed), one wave per 64 pixels and one pixel per lane, the
// mixture in registers across the frames of the launch, 64-pixel field-major
// record groups, and the same block-staged input as the cascade.
template <int C, int K, bool F32>
__global__ __launch_bounds__(64) void k_gmm(Buffers b, Frames fr, KParams kp) {
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t tile0 = tile * 64;
  const int64_t p = tile0 + lane;
  const bool valid = p < b.P;
  const int64_t rem = b.P - tile0;
  const int npx = rem >= 64 ? 64 : (int)rem;
  Mix<C, K> m;
  float x[C];
#pragma unroll
  for (int c = 0; c < C; ++c) x[c] = 0.0f;
  if (valid) grp_load<C, K>(b.gmm, p, m);
  bool lab = false;

  constexpr int NB = 8;
  using Stage = InStage<C, F32, NB>;
  __shared__ uint32_t s_in[NB * Stage::NDW * 64];
  Stage in;
  if (fr.nframes > 0) in.issue(fr.x, fr.stride, fr.nframes, 0, tile0, npx, lane);
  for (int f0 = 0; f0 < fr.nframes; f0 += NB) {
    in.commit(s_in, lane);
    wave_sync();
    in.issue(fr.x, fr.stride, fr.nframes, f0 + NB, tile0, npx, lane);
    const int nk = fr.nframes - f0 < NB ? fr.nframes - f0 : NB;
    for (int k = 0; k < nk; ++k) {
      const int f = f0 + k;
      Stage::read(s_in, k, frame_ptr<C, F32>(fr.x, fr.stride, f), tile0, lane, x);
      if (valid) {
        int l, mp;
        mix_step<C, K>(m, x, kp.alpha, kp, l, mp);
        lab = l != 0;
        if (fr.mask)
          __builtin_nontemporal_store((uint8_t)(lab ? 255 : 0), fr.mask + (int64_t)f * fr.mstride + p);
      }
      if (fr.partials) {
        const uint32_t nv = (uint32_t)__popcll(__ballot(valid));
        const uint32_t nf = (uint32_t)__popcll(__ballot(valid && lab));
        if (lane == 0) fr.partials[(int64_t)f * fr.nslots + tile] = stat_row(0u, 0u, 0u, nv, nv - nf, nf, 0u);
      }
    }
    wave_sync();
  }
  if (valid) {
    grp_store<C, K>(b.gmm, p, m);
    if (fr.nframes > 0) store_px<C, F32>(b.prev, p, x);
  }
  const unsigned long long bal = __ballot(lab);
  if (fr.nframes > 0 && lane == 0) b.labels[tile0 >> 6] = bal;
}

inline unsigned grid_for(int64_t P, int tile) { return (unsigned)((P + tile - 1) / tile); }

}  // namespace

// ---- launchers, one mixture size K per instantiation ---------------------------
#define COG_C_CASES(M, ...)                               \
  if (C == 3 && !f32in) { M(3, false, __VA_ARGS__); }     \
  else if (C == 3 && f32in) { M(3, true, __VA_ARGS__); }  \
  else if (C == 1 && !f32in) { M(1, false, __VA_ARGS__); } \
  else if (C == 1 && f32in) { M(1, true, __VA_ARGS__); }  \
  else return hipErrorInvalidValue;

template <int K>
hipError_t launch_train_k(int C, bool f32in, bool prior, const Buffers &b, const void *frames,
                          int64_t stride, int n, const KParams &kp, int64_t p0, int64_t p1,
                          hipStream_t s) {
  if (p1 <= p0) return hipSuccess;
  const int64_t np = p1 - p0;
  const unsigned g = grid_for(np, kNT);
#define COG_TRAIN(CC, FF, _)                                                                   \
  if (prior)                                                                                   \
    hipLaunchKernelGGL((k_train_prior<CC, K, FF>), dim3(grid_for(np, kTrainPx)),              \
                       dim3(2 * kTrainPx), 0, s, b, frames, stride, n, kp, p0, p1);            \
  else                                                                                         \
    hipLaunchKernelGGL((k_train<CC, K, FF>), dim3(g), dim3(kNT), 0, s, b, frames, stride, n, kp, \
                       p0, p1)
  COG_C_CASES(COG_TRAIN, 0)
#undef COG_TRAIN
  return hipGetLastError();
}

template <int K>
hipError_t launch_cascade_k(int C, bool f32in, int tile, const Buffers &b, const Frames &fr,
                            const KParams &kp, hipStream_t s) {
  const unsigned g = grid_for(b.P, tile);
  // the prior goes to LDS when a launch covers enough frames to amortise it
  const bool lp = fr.nframes >= 8;
  // sampling runs in the 64-pixel kernel only (the host rejects other tiles)
  const bool samp = (kp.stage_mask & 8u) != 0;
  if (samp && tile != 64) return hipErrorInvalidValue;
#define COG_CASC(CC, FF, PP, LL) \
  hipLaunchKernelGGL((k_cascade<CC, K, FF, PP, LL>), dim3(g), dim3(kNT), 0, s, b, fr, kp)
#define COG_CASCW(CC, FF, PP, LL) \
  hipLaunchKernelGGL((k_cascade_w<CC, K, FF, PP, LL>), dim3(g), dim3(64), 0, s, b, fr, kp)
#define COG_CASCD(CC, FF, LL, SS) \
  hipLaunchKernelGGL((k_cascade_d<CC, K, FF, LL, SS>), dim3(g), dim3(64), 0, s, b, fr, kp)
#define COG_CASC_TILE(CC, FF, _)                                            \
  switch (tile * 2 + (lp ? 1 : 0)) {                                        \
    case 128:                                                               \
      if (samp) COG_CASCD(CC, FF, false, true);                             \
      else COG_CASCD(CC, FF, false, false);                                 \
      break;                                                                \
    case 129:                                                               \
      if (samp) COG_CASCD(CC, FF, true, true);                              \
      else COG_CASCD(CC, FF, true, false);                                  \
      break;                                                                \
    case 256: COG_CASCW(CC, FF, 2, false); break;                           \
    case 257: COG_CASCW(CC, FF, 2, true); break;                            \
    case 512: COG_CASC(CC, FF, 1, false); break;                            \
    case 513: COG_CASC(CC, FF, 1, true); break;                             \
    case 1024: COG_CASC(CC, FF, 2, false); break;                           \
    case 1025: COG_CASC(CC, FF, 2, true); break;                            \
    case 2048: COG_CASC(CC, FF, 4, false); break;                           \
    case 2049: COG_CASC(CC, FF, 4, true); break;                            \
    default: return hipErrorInvalidValue;                                   \
  }
  COG_C_CASES(COG_CASC_TILE, 0)
#undef COG_CASC_TILE
#undef COG_CASCD
#undef COG_CASCW
#undef COG_CASC
  return hipGetLastError();
}

template <int K>
hipError_t launch_frame_k(int C, bool f32in, const Buffers &b, const Frames &fr, const KParams &kp,
                          hipStream_t s) {
  if (fr.nframes != 1 || (kp.stage_mask & 8u)) return hipErrorInvalidValue;
  const unsigned g = grid_for(b.P, kFrameTile);
#define COG_FRAME(CC, FF, _) \
  hipLaunchKernelGGL((k_frame<CC, K, FF>), dim3(g), dim3(64), 0, s, b, fr, kp)
  COG_C_CASES(COG_FRAME, 0)
#undef COG_FRAME
  return hipGetLastError();
}

template <int K>
hipError_t launch_tick_k(int C, bool f32in, bool lp, bool samp, TickHead *head,
                         const TickItem *items, int grid, int dynamic, hipStream_t s) {
  if (grid <= 0) return hipErrorInvalidValue;
#define COG_TICK(CC, FF, LL, SS) \
  hipLaunchKernelGGL((k_tick<CC, K, FF, LL, SS>), dim3(grid), dim3(64), 0, s, head, items, dynamic)
#define COG_TICK_LP(CC, FF, _)                   \
  if (lp) {                                      \
    if (samp) COG_TICK(CC, FF, true, true);      \
    else COG_TICK(CC, FF, true, false);          \
  } else {                                       \
    if (samp) COG_TICK(CC, FF, false, true);     \
    else COG_TICK(CC, FF, false, false);         \
  }
  COG_C_CASES(COG_TICK_LP, 0)
#undef COG_TICK_LP
#undef COG_TICK
  return hipGetLastError();
}

template <int K>
hipError_t launch_tick_c_k(int C, bool f32in, TickHead *head, const TickItem *items, int grid,
                           int dynamic, hipStream_t s) {
  if (grid <= 0) return hipErrorInvalidValue;
#define COG_TICKC(CC, FF, _) \
  hipLaunchKernelGGL((k_tick_c<CC, K, FF>), dim3(grid), dim3(64), 0, s, head, items, dynamic)
  COG_C_CASES(COG_TICKC, 0)
#undef COG_TICKC
  return hipGetLastError();
}

template <int K>
int tick_c_blocks_per_cu_k(int C, bool f32in) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  if (C == 3 && !f32in) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tick_c<3, K, false>, 64, 0);
  else if (C == 3 && f32in) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tick_c<3, K, true>, 64, 0);
  else if (C == 1 && !f32in) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tick_c<1, K, false>, 64, 0);
  else if (C == 1 && f32in) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tick_c<1, K, true>, 64, 0);
  return e == hipSuccess ? nb : 0;
}

template <int K>
int tick_blocks_per_cu_k(int C, bool f32in, bool lp, bool samp) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define COG_OCC(CC, FF, LL, SS) \
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tick<CC, K, FF, LL, SS>, 64, 0)
#define COG_OCC_LP(CC, FF, _)                   \
  if (lp) {                                     \
    if (samp) COG_OCC(CC, FF, true, true);      \
    else COG_OCC(CC, FF, true, false);          \
  } else {                                      \
    if (samp) COG_OCC(CC, FF, false, true);     \
    else COG_OCC(CC, FF, false, false);         \
  }
  if (C == 3 && !f32in) { COG_OCC_LP(3, false, 0) }
  else if (C == 3 && f32in) { COG_OCC_LP(3, true, 0) }
  else if (C == 1 && !f32in) { COG_OCC_LP(1, false, 0) }
  else if (C == 1 && f32in) { COG_OCC_LP(1, true, 0) }
#undef COG_OCC_LP
#undef COG_OCC
  return e == hipSuccess ? nb : 0;
}

template <int K>
hipError_t launch_gmm_k(int C, bool f32in, const Buffers &b, const Frames &fr, const KParams &kp,
                        hipStream_t s) {
  const unsigned g = grid_for(b.P, 64);
#define COG_GMM(CC, FF, _) \
  hipLaunchKernelGGL((k_gmm<CC, K, FF>), dim3(g), dim3(64), 0, s, b, fr, kp)
  COG_C_CASES(COG_GMM, 0)
#undef COG_GMM
  return hipGetLastError();
}

#undef COG_C_CASES

// Explicit instantiation of every launcher for one K.
#define COG_INSTANTIATE_K(KK)                                                                  \
  template hipError_t launch_train_k<KK>(int, bool, bool, const Buffers &, const void *,     \
                                         int64_t, int, const KParams &, int64_t, int64_t,      \
                                         hipStream_t);                                         \
  template hipError_t launch_cascade_k<KK>(int, bool, int, const Buffers &, const Frames &,   \
                                           const KParams &, hipStream_t);                      \
  template hipError_t launch_frame_k<KK>(int, bool, const Buffers &, const Frames &,           \
                                         const KParams &, hipStream_t);                        \
  template hipError_t launch_tick_k<KK>(int, bool, bool, bool, TickHead *, const TickItem *,   \
                                        int, int, hipStream_t);                                \
  template int tick_blocks_per_cu_k<KK>(int, bool, bool, bool);                                \
  template hipError_t launch_tick_c_k<KK>(int, bool, TickHead *, const TickItem *, int, int,   \
                                          hipStream_t);                                        \
  template int tick_c_blocks_per_cu_k<KK>(int, bool);                                          \
  template hipError_t launch_gmm_k<KK>(int, bool, const Buffers &, const Frames &,             \
                                       const KParams &, hipStream_t);

}  // namespace cog
