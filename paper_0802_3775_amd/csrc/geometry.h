// Host-side geometry helpers of libfdtd (see geometry.cpp).
#pragma once
#include <cstdint>
#include <vector>

namespace fdg {

struct OpalSpec {
  int cells[3];
  int periodic[3];
  int res;
  double r0;
  int disorder;     // 0 none, 1 uniform radius, 2 Gaussian jitter
  double strength;
  uint32_t seed, realization;
};

void philox4x32_10(const uint32_t in[4], uint32_t k0, uint32_t k1, uint32_t out[4]);
void normals4(const uint32_t ctr[4], uint32_t k0, uint32_t k1, double g[4]);
// rows of (site id, Cx, Cy, Cz, rho) in quanta a/(2 res 2^16), crystal-relative
int build_spheres(const OpalSpec& o, std::vector<int64_t>& rows);

}  // namespace fdg
