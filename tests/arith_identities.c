/* Exhaustive host checks of two arithmetic identities that the GPU kernels
 * rely on (paper_1805_06019_amd/csrc/kernels.hip), restated here in plain C:
 *
 * 1. unzigzag_pk: two zigzagged values (0, 1, 2, 3, ... -> 0, -1, 1, -2, ...,
 *    Sec. 3.2) in the 16-bit halves of a word, undone and multiplied by 2^q
 *    with one right rotation by (33 - q) mod 32 (the kernels' alignbit of the
 *    word with itself), a mask that clears each half's top bit, and a
 *    multiply that inverts a negative value's bits from q - 1 up.  Checked
 *    against the definition, per half, for every pair of zigzag values below
 *    2^12 (a valid stream holds no larger one) and every q = 0..4.
 *
 * 2. div255: x / 255 as the product with the rounded reciprocal, corrected by
 *    one fused residual step.  Checked against the IEEE single-precision
 *    quotient for every float in [0, 255] (the interpolation only divides
 *    lerps of 8-bit samples).
 *
 * Prints one line per identity ("<name>: <cases> cases, <n> differ"); exit
 * status 0 when neither differs anywhere.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

static uint32_t rotr32(uint32_t x, unsigned s) {
  s &= 31u;
  return s ? (x >> s) | (x << (32u - s)) : x;
}

static uint32_t unzigzag_pk(uint32_t z, int q) {
  const uint32_t rot = (uint32_t)(33 - q) & 31u;
  const uint32_t inv = q ? (0xFFFFu << (q - 1)) & 0xFFFFu : 0xFFFFu;
  const uint32_t t = rotr32(z, rot) & 0x7FFF7FFFu;
  return t ^ ((z & 0x00010001u) * inv);
}

/* the definition, one value: even z -> z / 2, odd z -> -(z + 1) / 2; times 2^q as int16 */
static uint16_t unzigzag_ref(uint32_t z, int q) {
  const int32_t v = (z & 1u) ? -(int32_t)((z + 1u) >> 1) : (int32_t)(z >> 1);
  return (uint16_t)(int16_t)(v * (1 << q));
}

static float div255(float x) {
  const float r = 1.0f / 255.0f;
  const float q = x * r;
  return fmaf(fmaf(-q, 255.0f, x), r, q);
}

int main(void) {
  long long zz_cases = 0, zz_bad = 0;
  for (int q = 0; q <= 4; q++) {
#pragma omp parallel for reduction(+ : zz_cases, zz_bad)
    for (uint32_t lo = 0; lo < 4096u; lo++)
      for (uint32_t hi = 0; hi < 4096u; hi++) {
        const uint32_t z = lo | hi << 16;
        const uint32_t want = (uint32_t)unzigzag_ref(lo, q) | (uint32_t)unzigzag_ref(hi, q) << 16;
        zz_bad += unzigzag_pk(z, q) != want;
        zz_cases++;
      }
  }
  printf("unzigzag_pk: %lld cases, %lld differ\n", zz_cases, zz_bad);

  float top = 255.0f;
  uint32_t top_bits;
  memcpy(&top_bits, &top, 4);
  long long dv_cases = 0, dv_bad = 0;
  /* the non-negative floats up to 255, in increasing order of their bit patterns
     (dynamic chunks: the host's arithmetic on subnormals at the low end is slow) */
#pragma omp parallel for schedule(dynamic, 1 << 20) reduction(+ : dv_cases, dv_bad)
  for (long long u = 0; u <= (long long)top_bits; u++) {
    const uint32_t b = (uint32_t)u;
    float x;
    memcpy(&x, &b, 4);
    const float got = div255(x), want = x / 255.0f;
    uint32_t gb, wb;
    memcpy(&gb, &got, 4);
    memcpy(&wb, &want, 4);
    dv_bad += gb != wb;
    dv_cases++;
  }
  printf("div255: %lld cases, %lld differ\n", dv_cases, dv_bad);
  return (zz_bad || dv_bad) ? 1 : 0;
}
