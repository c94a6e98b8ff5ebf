// Host-side geometry of libfdtd: Philox4x32-10, Box-Muller normals and the
// quantized sphere list of an inverted opal (FP64, then exact integers).
//
// Paper (arXiv:0802.3775), section "Sample and numerical approach": air
// spheres at the fcc sites of a cubic lattice in a dielectric background,
// r0 = a/(2 sqrt 2); disorder r = r0 (1 + gamma xi), xi uniform in [-1/2, 1/2].
// Gaussian jitter of radius and centre with deviation delta (truncated at
// +-4 delta, radius clipped at 0) is the second disorder model.
//
// Definitions fixed by this library's contract (the voxel maps must be
// reproducible bit for bit anywhere):
//   uniform  u = ((x >> 8) + 1/2) 2^-24 from a Philox word x;
//   normals  (sqrt(-2 ln u1) cos(2 pi u2), sqrt(-2 ln u1) sin(2 pi u2)) from
//            the pairs (word0, word1) and (word2, word3);
//   counter  (site id, 0, 0, 0), key (seed, realization);
//   quanta   q = a / (2 res 2^16); centre and radius rounded to nearest, ties
//            to even.
#include <cmath>
#include <cstdint>
#include <vector>

#include "geometry.h"

namespace fdg {

void philox4x32_10(const uint32_t in[4], uint32_t k0, uint32_t k1, uint32_t out[4]) {
  uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u24(uint32_t x) { return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0); }

void normals4(const uint32_t ctr[4], uint32_t k0, uint32_t k1, double g[4]) {
  uint32_t w[4];
  philox4x32_10(ctr, k0, k1, w);
  const double two_pi = 6.283185307179586476925286766559;
  for (int h = 0; h < 2; ++h) {
    const double radius = std::sqrt(-2.0 * std::log(u24(w[2 * h])));
    const double ang = two_pi * u24(w[2 * h + 1]);
    g[2 * h] = radius * std::cos(ang);
    g[2 * h + 1] = radius * std::sin(ang);
  }
}

int build_spheres(const OpalSpec& o, std::vector<int64_t>& rows) {
  rows.clear();
  int64_t ext[3];
  for (int a = 0; a < 3; ++a) {
    if (o.cells[a] < 1) return -1;
    ext[a] = 2 * (int64_t)o.cells[a] + (o.periodic[a] ? 0 : 1);
  }
  const int64_t wx = 2 * (int64_t)o.cells[0] + 1, wy = 2 * (int64_t)o.cells[1] + 1;
  const double scale = 2.0 * (double)o.res * 65536.0;
  for (int64_t l = 0; l < ext[2]; ++l)
    for (int64_t k = 0; k < ext[1]; ++k)
      for (int64_t h = 0; h < ext[0]; ++h) {
        if ((h + k + l) % 2 != 0) continue;
        const int64_t id = h + wx * (k + wy * l);
        double centre[3] = {0.5 * (double)h, 0.5 * (double)k, 0.5 * (double)l};
        double radius = o.r0;
        const uint32_t ctr[4] = {(uint32_t)id, 0u, 0u, 0u};
        if (o.disorder == 1) {
          uint32_t w[4];
          philox4x32_10(ctr, o.seed, o.realization, w);
          const double xi = u24(w[0]) - 0.5;
          radius = o.r0 * (1.0 + o.strength * xi);
        } else if (o.disorder == 2) {
          double g[4];
          normals4(ctr, o.seed, o.realization, g);
          for (double& v : g) v = v > 4.0 ? 4.0 : (v < -4.0 ? -4.0 : v);
          radius = o.r0 + o.strength * g[0];
          for (int a = 0; a < 3; ++a) centre[a] = centre[a] + o.strength * g[1 + a];
        }
        if (radius < 0.0) radius = 0.0;
        rows.push_back(id);
        for (int a = 0; a < 3; ++a) rows.push_back((int64_t)std::nearbyint(centre[a] * scale));
        rows.push_back((int64_t)std::nearbyint(radius * scale));
      }
  return 0;
}

}  // namespace fdg
