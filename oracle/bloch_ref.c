/*
 * FP64 density-matrix gain model of the oracle (test infrastructure only).
 * The equations and the time splitting are stated in bloch_ref.h.  The
 * coherent propagator is formed by a plain complex Gauss-Jordan solve of
 * (I + i tau H') V = (I - i tau H') and applied as V rho V^+ with full 4x4
 * products: no use is made of the structure of H.
 */
#include <math.h>
#include <string.h>
#include "bloch_ref.h"

#define PI 3.141592653589793238462643383279502884
#define C_LIGHT 299792458.0
#define EPS0 8.8541878128e-12
#define HBAR 1.054571817e-34

int orc_bloch_setup(const orc_material* m, double dt, double dx, double a_meters, orc_bloch_c* c) {
  if (!(m->f_a > 0.0) || !(m->t1 > 0.0) || !(m->t2 > 0.0) || m->n_total < 0.0 || m->pump < 0.0 ||
      !(m->eps > 0.0) || !(a_meters > 0.0))
    return -1;
  const double t_unit = a_meters / C_LIGHT;
  c->w0 = 2.0 * PI * m->f_a;
  if (!(c->w0 * dt < PI)) return -1;
  c->wp = (2.0 / dt) * tan(0.5 * c->w0 * dt);
  /* dipole moment: given, or the radiative-limit value that makes T1 the
     spontaneous lifetime in a host of index sqrt(eps) */
  double mu = m->dipole;
  if (!(mu > 0.0)) {
    const double w_si = c->w0 * C_LIGHT / a_meters;
    mu = sqrt(3.0 * PI * EPS0 * HBAR * C_LIGHT * C_LIGHT * C_LIGHT /
              (w_si * w_si * w_si * sqrt(m->eps) * m->t1));
  }
  c->kappa = m->n_total * mu * mu * a_meters / (EPS0 * HBAR * C_LIGHT);
  c->g1 = t_unit / m->t1;
  c->g2 = t_unit / m->t2;
  c->gp = m->pump * t_unit;
  c->noise = m->noise / sqrt(dt * dx * dx * dx);
  return 0;
}

void orc_bloch_relax(const orc_bloch_c* c, double tau, orc_z r[4][4]) {
  double e = 0.0;
  for (int k = 1; k < 4; ++k) e += creal(r[k][k]);
  const double rate = c->gp + c->g1;
  double e_new = e;
  if (rate > 0.0) {
    const double e_inf = c->gp / rate;
    e_new = e_inf + (e - e_inf) * exp(-rate * tau);
  }
  const double h1 = exp(-c->g1 * tau);
  for (int k = 1; k < 4; ++k) r[k][k] = e_new / 3.0 + (creal(r[k][k]) - e / 3.0) * h1;
  r[0][0] = creal(r[0][0]) - (e_new - e);
  const double h2 = exp(-c->g2 * tau);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      if (a != b) r[a][b] *= h2;
}

/* Solve A X = B for 4x4 complex matrices (Gauss-Jordan, partial pivoting). */
static void solve4(orc_z A[4][4], orc_z B[4][4], orc_z X[4][4]) {
  orc_z W[4][8];
  for (int r = 0; r < 4; ++r)
    for (int q = 0; q < 4; ++q) {
      W[r][q] = A[r][q];
      W[r][q + 4] = B[r][q];
    }
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (cabs(W[r][col]) > cabs(W[piv][col])) piv = r;
    for (int q = 0; q < 8; ++q) {
      orc_z t = W[col][q];
      W[col][q] = W[piv][q];
      W[piv][q] = t;
    }
    const orc_z inv = 1.0 / W[col][col];
    for (int q = 0; q < 8; ++q) W[col][q] *= inv;
    for (int r = 0; r < 4; ++r) {
      if (r == col) continue;
      const orc_z f = W[r][col];
      for (int q = 0; q < 8; ++q) W[r][q] -= f * W[col][q];
    }
  }
  for (int r = 0; r < 4; ++r)
    for (int q = 0; q < 4; ++q) X[r][q] = W[r][q + 4];
}

void orc_bloch_coherent(const orc_bloch_c* c, double dt, const double E[3], orc_z r[4][4]) {
  orc_z H[4][4];
  memset(H, 0, sizeof(H));
  for (int k = 1; k < 4; ++k) {
    H[k][k] = c->wp;
    H[0][k] = -E[k - 1];
    H[k][0] = -E[k - 1];
  }
  const double tau = 0.5 * dt;
  orc_z Ap[4][4], Am[4][4], V[4][4], T[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const orc_z id = a == b ? 1.0 : 0.0;
      Ap[a][b] = id + I * tau * H[a][b];
      Am[a][b] = id - I * tau * H[a][b];
    }
  solve4(Ap, Am, V);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      orc_z acc = 0.0;
      for (int q = 0; q < 4; ++q) acc += V[a][q] * r[q][b];
      T[a][b] = acc;
    }
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      orc_z acc = 0.0;
      for (int q = 0; q < 4; ++q) acc += T[a][q] * conj(V[b][q]);
      r[a][b] = acc;
    }
}

void orc_bloch_step(const orc_bloch_c* c, double dt, const double E[3], orc_z in[4][4], orc_z out[4][4]) {
  memcpy(out, in, sizeof(orc_z) * 16);
  orc_bloch_relax(c, 0.5 * dt, out);
  orc_bloch_coherent(c, dt, E, out);
  orc_bloch_relax(c, 0.5 * dt, out);
}

/* Matter alone: nsteps of S(rho; emid[n]) from rho (32 doubles: row-major 4x4,
   (re, im) pairs), keeping the state after each step in hist (nsteps x 32) when
   hist is not NULL. */
int orc_bloch_evolve(const orc_material* m, double dt, double dx, double a_meters, int64_t nsteps,
                     const double* emid, double* rho, double* hist) {
  orc_bloch_c c;
  if (m->gain != 2 || orc_bloch_setup(m, dt, dx, a_meters, &c)) return -1;
  orc_z r[4][4], o[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) r[a][b] = rho[2 * (4 * a + b)] + I * rho[2 * (4 * a + b) + 1];
  for (int64_t n = 0; n < nsteps; ++n) {
    orc_bloch_step(&c, dt, emid + 3 * n, r, o);
    memcpy(r, o, sizeof(r));
    if (hist)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          hist[32 * n + 2 * (4 * a + b)] = creal(r[a][b]);
          hist[32 * n + 2 * (4 * a + b) + 1] = cimag(r[a][b]);
        }
  }
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      rho[2 * (4 * a + b)] = creal(r[a][b]);
      rho[2 * (4 * a + b) + 1] = cimag(r[a][b]);
    }
  return 0;
}

/* Constants of the model for material m (w0, w', kappa, 1/T1, 1/T2, pump). */
int orc_bloch_constants(const orc_material* m, double dt, double dx, double a_meters, double* out6) {
  orc_bloch_c c;
  if (m->gain != 2 || orc_bloch_setup(m, dt, dx, a_meters, &c)) return -1;
  out6[0] = c.w0; out6[1] = c.wp; out6[2] = c.kappa;
  out6[3] = c.g1; out6[4] = c.g2; out6[5] = c.gp;
  return 0;
}
