/*
 * Inverted-opal geometry for the oracle (test infrastructure only).
 *
 * Paper, section "Sample and numerical approach": the photonic crystal is an
 * inverted opal, air spheres at the sites of an fcc lattice (cubic lattice
 * constant a) in a dielectric background; the ordered radius is r0 = a/(2 sqrt 2);
 * disorder sets each radius to r0 (1 + gamma xi) with xi uniform in [-1/2, 1/2].
 * A second disorder model jitters radii and centres with Gaussian deviates of
 * standard deviation delta (reading; truncated at 4 delta, radius clipped at 0).
 *
 * Integer contract (reading): with quantum q = a / (2 res 2^16), sphere centres
 * and radii are rounded to the nearest integer multiple of q (ties to even);
 * a voxel centre sits at (2 (i - origin) + 1) 2^16 quanta; a voxel lies inside a
 * sphere iff the squared integer distance is strictly less than rho^2.
 * Periodic axes use the minimum image.  A voxel is "void" iff it lies inside
 * the crystal region and inside any sphere.
 *
 * Sites: (h, k, l)/2 with h + k + l even; each index runs over [0, 2n) on a
 * periodic axis and [0, 2n] on a closed axis.  Site id = h + (2nx+1)(k + (2ny+1) l).
 * Draws: Philox key (seed, realization), counter (id, 0, 0, 0).
 *
 * Two voxelizers are kept on purpose: a per-voxel gather over all spheres and a
 * per-sphere scatter over each sphere's bounding box.  They must agree bit for
 * bit; the tests check that.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static const int64_t HALF_VOXEL = 65536; /* 2^16 quanta = dx/2 */

static int64_t site_extent(const orc_grid* g, const orc_opal* o, int d) {
  return g->periodic[d] ? 2 * (int64_t)o->cells[d] : 2 * (int64_t)o->cells[d] + 1;
}

static int check_opal(const orc_grid* g, const orc_opal* o) {
  const int32_t n[3] = {g->nx, g->ny, g->nz};
  for (int d = 0; d < 3; ++d) {
    if (o->cells[d] < 1 || o->origin[d] < 0) return -1;
    if ((int64_t)o->origin[d] + (int64_t)o->cells[d] * g->res > n[d]) return -1;
    if (g->periodic[d] && (o->origin[d] != 0 || o->cells[d] * g->res != n[d])) return -1;
  }
  return 0;
}

int64_t orc_opal_count(const orc_grid* g, const orc_opal* o) {
  if (check_opal(g, o)) return -1;
  int64_t count = 0;
  for (int64_t l = 0; l < site_extent(g, o, 2); ++l)
    for (int64_t k = 0; k < site_extent(g, o, 1); ++k)
      for (int64_t h = 0; h < site_extent(g, o, 0); ++h)
        if (((h + k + l) & 1) == 0) ++count;
  return count;
}

int orc_opal_spheres(const orc_grid* g, const orc_opal* o, int64_t* out) {
  if (check_opal(g, o)) return -1;
  const double scale = 2.0 * (double)g->res * 65536.0; /* quanta per a */
  const uint32_t key[2] = {g->seed, g->realization};
  const int64_t ex = site_extent(g, o, 0), ey = site_extent(g, o, 1), ez = site_extent(g, o, 2);
  const int64_t wx = 2 * (int64_t)o->cells[0] + 1, wy = 2 * (int64_t)o->cells[1] + 1;
  int64_t row = 0;
  for (int64_t l = 0; l < ez; ++l)
    for (int64_t k = 0; k < ey; ++k)
      for (int64_t h = 0; h < ex; ++h) {
        if ((h + k + l) & 1) continue;
        int64_t id = h + wx * (k + wy * l);
        double c[3] = {0.5 * (double)h, 0.5 * (double)k, 0.5 * (double)l};
        double r = o->r0;
        if (o->disorder != ORC_DIS_NONE) {
          uint32_t ctr[4] = {(uint32_t)id, 0u, 0u, 0u};
          if (o->disorder == ORC_DIS_UNIFORM_RADIUS) {
            uint32_t raw[4];
            orc_philox4x32_10(ctr, key, raw);
            double xi = ((double)(raw[0] >> 8) + 0.5) * (1.0 / 16777216.0) - 0.5;
            r = o->r0 * (1.0 + o->strength * xi);
          } else {
            double gs[4];
            orc_normals4(ctr, key, gs);
            for (int q = 0; q < 4; ++q) {
              if (gs[q] > 4.0) gs[q] = 4.0;
              if (gs[q] < -4.0) gs[q] = -4.0;
            }
            r = o->r0 + o->strength * gs[0];
            for (int d = 0; d < 3; ++d) c[d] = c[d] + o->strength * gs[1 + d];
          }
        }
        if (r < 0.0) r = 0.0;
        out[5 * row + 0] = id;
        out[5 * row + 1] = (int64_t)nearbyint(c[0] * scale);
        out[5 * row + 2] = (int64_t)nearbyint(c[1] * scale);
        out[5 * row + 3] = (int64_t)nearbyint(c[2] * scale);
        out[5 * row + 4] = (int64_t)nearbyint(r * scale);
        ++row;
      }
  return 0;
}

/* Displacement along one axis, minimum image when periodic. */
static int64_t axis_delta(int64_t x, int64_t c, int periodic, int64_t period) {
  int64_t d = x - c;
  if (periodic) {
    d %= period;
    if (d < 0) d += period;
    if (2 * d > period) d -= period;
  }
  return d;
}

static int inside_crystal(const orc_opal* o, int32_t res, int64_t i, int64_t j, int64_t k) {
  const int64_t p[3] = {i, j, k};
  for (int d = 0; d < 3; ++d)
    if (p[d] < o->origin[d] || p[d] >= o->origin[d] + (int64_t)o->cells[d] * res) return 0;
  return 1;
}

static int check_spheres(const orc_grid* g, const orc_opal* o, const int64_t* sph, int64_t n) {
  for (int d = 0; d < 3; ++d) {
    if (!g->periodic[d]) continue;
    int64_t period = (int64_t)o->cells[d] * g->res * 2 * HALF_VOXEL;
    for (int64_t s = 0; s < n; ++s)
      if (2 * sph[5 * s + 4] >= period) return -1; /* minimum image would be ambiguous */
  }
  return 0;
}

int orc_voxelize_gather(const orc_grid* g, const orc_opal* o, const int64_t* sph, int64_t n,
                        uint8_t* map) {
  if (check_opal(g, o) || check_spheres(g, o, sph, n)) return -1;
  const int64_t nx = g->nx, ny = g->ny, nz = g->nz;
  int64_t period[3];
  for (int d = 0; d < 3; ++d) period[d] = (int64_t)o->cells[d] * g->res * 2 * HALF_VOXEL;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        uint8_t m;
        if (!inside_crystal(o, g->res, i, j, k)) {
          m = (uint8_t)o->mat_out;
        } else {
          int64_t X[3] = {(2 * (i - o->origin[0]) + 1) * HALF_VOXEL,
                          (2 * (j - o->origin[1]) + 1) * HALF_VOXEL,
                          (2 * (k - o->origin[2]) + 1) * HALF_VOXEL};
          int hit = 0;
          for (int64_t s = 0; s < n && !hit; ++s) {
            int64_t r2 = 0;
            for (int d = 0; d < 3; ++d) {
              int64_t dd = axis_delta(X[d], sph[5 * s + 1 + d], g->periodic[d], period[d]);
              r2 += dd * dd;
            }
            if (r2 < sph[5 * s + 4] * sph[5 * s + 4]) hit = 1;
          }
          m = (uint8_t)(hit ? o->mat_void : o->mat_bg);
        }
        map[(k * ny + j) * nx + i] = m;
      }
  return 0;
}

/* floor(a / b) for b > 0 */
static int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && (a < 0)) --q;
  return q;
}

int orc_voxelize_scatter(const orc_grid* g, const orc_opal* o, const int64_t* sph, int64_t n,
                         uint8_t* map) {
  if (check_opal(g, o) || check_spheres(g, o, sph, n)) return -1;
  const int64_t nx = g->nx, ny = g->ny, nz = g->nz;
  const int64_t ncr[3] = {(int64_t)o->cells[0] * g->res, (int64_t)o->cells[1] * g->res,
                          (int64_t)o->cells[2] * g->res};
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i)
        map[(k * ny + j) * nx + i] =
            (uint8_t)(inside_crystal(o, g->res, i, j, k) ? o->mat_bg : o->mat_out);
  for (int64_t s = 0; s < n; ++s) {
    const int64_t* S = sph + 5 * s;
    const int64_t rho = S[4];
    if (rho <= 0) continue;
    /* crystal-relative voxel index range whose centres can fall within rho */
    int64_t lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = floordiv(S[1 + d] - rho, 2 * HALF_VOXEL) - 1;
      hi[d] = floordiv(S[1 + d] + rho, 2 * HALF_VOXEL) + 1;
      if (!g->periodic[d]) {
        if (lo[d] < 0) lo[d] = 0;
        if (hi[d] > ncr[d] - 1) hi[d] = ncr[d] - 1;
      }
    }
    for (int64_t c = lo[2]; c <= hi[2]; ++c)
      for (int64_t b = lo[1]; b <= hi[1]; ++b)
        for (int64_t a = lo[0]; a <= hi[0]; ++a) {
          int64_t rel[3] = {a, b, c};
          int64_t r2 = 0;
          for (int d = 0; d < 3; ++d) {
            /* unwrapped centre minus sphere centre; on periodic axes the box never
               spans more than one period, so the unwrapped delta is the minimum image
               of some voxel; fold the index back into the crystal */
            int64_t dd = (2 * rel[d] + 1) * HALF_VOXEL - S[1 + d];
            r2 += dd * dd;
          }
          if (r2 >= rho * rho) continue;
          int64_t idx[3];
          for (int d = 0; d < 3; ++d) {
            int64_t w = rel[d];
            if (g->periodic[d]) {
              w %= ncr[d];
              if (w < 0) w += ncr[d];
            }
            idx[d] = w + o->origin[d];
          }
          map[(idx[2] * ny + idx[1]) * nx + idx[0]] = (uint8_t)o->mat_void;
        }
  }
  return 0;
}
