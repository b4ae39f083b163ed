/*
 * rmat_draws.c -- the quadrant draws of the seeded R-MAT generator in
 * graphgen.py, written out in C because the NumPy form takes about a minute
 * at 2^22 vertices.  Input generation only: no shortest paths, path counts
 * or dependencies.  The output is bit-identical to graphgen's NumPy path
 * (a CPU test compares the two):
 *   draw e, bit level l (most significant first) reads value e*scale + l of
 *   the SplitMix64 stream `seed` (Steele, Lea and Flood 2014: value i is
 *   mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)), turns it into the double
 *   u = (x >> 11) * 2^-53 and picks the quadrant by the thresholds
 *   t1 = a, t2 = a + b, t3 = a + b + c: source bit (u >= t2), destination
 *   bit (t1 <= u < t2 or u >= t3).
 */
#include <stdint.h>

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* src[e], dst[e] for e in [0, ne): vertex ids of draw e before relabelling. */
void rmat_draws(uint64_t seed, int scale, int64_t ne, double t1, double t2, double t3, int64_t *src,
                int64_t *dst) {
  const uint64_t gamma = 0x9E3779B97F4A7C15ULL;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < ne; ++e) {
    int64_t s = 0, d = 0;
    uint64_t i = (uint64_t)e * (uint64_t)scale;
    for (int l = 0; l < scale; ++l, ++i) {
      const uint64_t x = mix64(seed + (i + 1) * gamma);
      const double u = (double)(x >> 11) * 0x1.0p-53;
      s = (s << 1) | (u >= t2);
      d = (d << 1) | ((u >= t1 && u < t2) || u >= t3);
    }
    src[e] = s;
    dst[e] = d;
  }
}
