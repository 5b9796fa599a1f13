/*
 * Seeded synthetic inputs for the closed-shell RI-MP2 fragment kernel.
 *
 * This file holds only random-number generation and input scaling; it contains
 * none of the MP2 arithmetic.  It feeds both the CPU oracle (through tests) and
 * the HIP path (through the benchmark and tests), so both see bit-identical
 * inputs.
 *
 * Generator (counter-based, so any slice can be regenerated independently):
 *   mix64(z)       : the SplitMix64 output function of Steele, Lea and Flood
 *                    ("Fast splittable pseudorandom number generators", 2014).
 *   draw(key, n)   = mix64(key + (n + 1) * GOLDEN)   -- the n-th SplitMix64
 *                    output of a generator whose state starts at key.
 *   key(seed, frag, tensor) = draw(draw(draw(seed, 0) ^ frag, 0) ^ tensor, 0)
 *   uniform(x)     = ((x >> 11) + 0.5) * 2^-53, strictly inside (0, 1)
 *   normal(key, e) = sqrt(-2 ln u1) * cos(2 pi u2) with u1 = uniform(draw(key, 2e)),
 *                    u2 = uniform(draw(key, 2e + 1))  (Box and Muller, 1958).
 * Elements are computed independently, so the result does not depend on the
 * number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL
#define TWO_PI 6.283185307179586

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t draw(uint64_t key, uint64_t n) { return mix64(key + (n + 1) * GOLDEN); }
static inline double uniform01(uint64_t x) { return ((double)(x >> 11) + 0.5) * 0x1.0p-53; }

uint64_t synth_key(uint64_t seed, uint64_t frag, uint64_t tensor) {
  return draw(draw(draw(seed, 0) ^ frag, 0) ^ tensor, 0);
}

uint64_t synth_draw(uint64_t key, uint64_t n) { return draw(key, n); }

static inline double normal_at(uint64_t key, uint64_t e) {
  double u1 = uniform01(draw(key, 2 * e)), u2 = uniform01(draw(key, 2 * e + 1));
  return sqrt(-2.0 * log(u1)) * cos(TWO_PI * u2);
}

/* out[n] = uniform(draw(key, first + n)) for n < count */
void synth_uniform(uint64_t key, uint64_t first, int64_t count, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < count; ++n) out[n] = uniform01(draw(key, first + (uint64_t)n));
}

/* out[n] = normal(key, first + n) for n < count */
void synth_normal(uint64_t key, uint64_t first, int64_t count, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < count; ++n) out[n] = normal_at(key, first + (uint64_t)n);
}

/*
 * Three-index tensor rows i in [i0, i1) of a [nocc][nvir][naux] tensor:
 *   out[(i - i0)][a][P] = normal(key, (i*nvir + a)*naux + P) * scale[s(i)][P]
 * where s(i) = i when scale_per_i is nonzero (scale is [nocc][naux]) and 0
 * otherwise (scale is one row of naux values).
 */
void synth_three_index(uint64_t key, int64_t i0, int64_t i1, int64_t nvir, int64_t naux,
                       const double* scale, int scale_per_i, double* out) {
  int64_t rows = (i1 - i0) * nvir;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r) {
    int64_t i = i0 + r / nvir;
    const double* sc = scale + (scale_per_i ? i * naux : 0);
    uint64_t e0 = (uint64_t)((i0 * nvir + r) * naux);
    double* o = out + r * naux;
    for (int64_t P = 0; P < naux; ++P) o[P] = normal_at(key, e0 + (uint64_t)P) * sc[P];
  }
}
