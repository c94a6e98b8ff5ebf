/*
 * Counter-based random numbers for the oracle (test infrastructure only).
 *
 * Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11): a 4 x 32-bit counter and a 2 x 32-bit
 * key; each of the ten rounds multiplies two counter words by the constants
 * 0xD2511F53 and 0xCD9E8D57 into 64-bit products, crosses the high halves with
 * the other two words and the key, and the key is bumped by the Weyl constants
 * 0x9E3779B9 and 0xBB67AE85 between rounds.
 *
 * Uniforms: u = (top 24 bits + 1/2) * 2^-24, exact in binary32 and binary64,
 * in (0, 1).  Normals: Box-Muller on the pairs (u0, u1) and (u2, u3).
 *
 * The paper draws its disorder with "a random-number generator" (section
 * "Sample and numerical approach") and adds spontaneous-emission noise as a
 * stochastic source; it does not name a generator.  Philox keyed by
 * (seed, realization) is this implementation's reading.
 */
#include <math.h>
#include <stdint.h>
#include "oracle.h"

static void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(0xD2511F53u, x0, &hi0, &lo0);
    mulhilo32(0xCD9E8D57u, x2, &hi1, &lo1);
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static double uniform24(uint32_t x) {
  return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0);
}

void orc_normals4(const uint32_t ctr[4], const uint32_t key[2], double g[4]) {
  uint32_t r[4];
  orc_philox4x32_10(ctr, key, r);
  const double two_pi = 6.283185307179586476925286766559;
  for (int p = 0; p < 2; ++p) {
    double u1 = uniform24(r[2 * p]);
    double u2 = uniform24(r[2 * p + 1]);
    double rad = sqrt(-2.0 * log(u1));
    g[2 * p] = rad * cos(two_pi * u2);
    g[2 * p + 1] = rad * sin(two_pi * u2);
  }
}
