/* Checks the reciprocal-based quotient the cascade kernels use in place of a
 * division (quot_recip): q = a y, then twice q <- q + (a - d q) y with fused
 * multiply-adds, y = 1/d correctly rounded.  Compared bit for bit with the
 * binary32 division:
 *   - every integer dividend of the scene-prior probability (0 .. 255^3 over
 *     255^3, and 0 .. 255 over 255), exhaustively;
 *   - the integer frame differences 0 .. 255 over divisors drawn across
 *     [2^-20, 2^20] (with all-ones and near-power-of-two significands);
 *   - dividends across [2^-100, 2^60] (either sign) over divisors across
 *     [2^-20, 2^20], random and edge significands;
 *   - mixture weights in [0, 1] over sums in [0.01, 2].
 * Prints the number of differing cases per group; argv[1] scales the random
 * groups. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static float quot_recip(float a, float d, float y) {
  const float q0 = a * y;
  const float q1 = fmaf(fmaf(-d, q0, a), y, q0);
  return fmaf(fmaf(-d, q1, a), y, q1);
}

static uint64_t st = 0x9e3779b97f4a7c15ull;
static uint64_t next(void) {
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return st;
}
static float from_bits(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static uint32_t bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static int same(float a, float d, float y) { return bits(quot_recip(a, d, y)) == bits(a / d); }

int main(int argc, char **argv) {
  const long scale = argc > 1 ? atol(argv[1]) : 1;
  long bad = 0;
  const float t3 = 16581375.0f, t1 = 255.0f;
  for (uint32_t p = 0; p <= 16581375u; ++p) bad += !same((float)p, t3, 1.0f / t3);
  for (uint32_t p = 0; p <= 255u; ++p) bad += !same((float)p, t1, 1.0f / t1);
  printf("prior %ld\n", bad);

  bad = 0;
  for (long i = 0; i < 20000 * scale; ++i) {
    uint32_t m = (uint32_t)(next() & 0x7fffff);
    if (i < 64) m = (i & 1) ? 0x7fffffu - (uint32_t)(i >> 1) : (uint32_t)(i >> 1);
    const float d = from_bits(((107u + (uint32_t)(next() % 41)) << 23) | m);
    const float y = 1.0f / d;
    for (int k = 0; k <= 255; ++k) bad += !same((float)k, d, y);
  }
  printf("difference %ld\n", bad);

  bad = 0;
  for (long i = 0; i < 4000000 * scale; ++i) {
    const uint64_t r = next();
    uint32_t ma = (uint32_t)(r >> 16) & 0x7fffff, md = (uint32_t)(next() & 0x7fffff);
    switch ((r >> 40) & 7) {
      case 0: ma = 0x7fffffu - (ma & 15); break;
      case 1: md = 0x7fffffu - (md & 15); break;
      case 2: md &= 15; break;
      case 3: ma &= 15; break;
      default: break;
    }
    float a = from_bits(((27u + (uint32_t)(r % 161)) << 23) | ma);
    const float d = from_bits(((107u + (uint32_t)((r >> 8) % 41)) << 23) | md);
    if (r >> 63) a = -a;
    bad += !same(a, d, 1.0f / d);
  }
  printf("general %ld\n", bad);

  bad = 0;
  for (long i = 0; i < 2000000 * scale; ++i) {
    const float S = 0.01f + (float)(next() >> 40) * 0x1p-24f * 1.99f;
    float w = (float)(next() >> 40) * 0x1p-24f;
    if (i & 1) w = w * S;
    bad += !same(w, S, 1.0f / S);
  }
  printf("weights %ld\n", bad);
  return 0;
}
