/*
 * FP64 density-matrix gain model of the oracle (test infrastructure only; see
 * oracle.h).  Internal to the oracle library.
 *
 * The paper's matter model (section "Sample and numerical approach"): a
 * four-level system whose three degenerate upper levels |1>, |2>, |3> couple
 * to Ex, Ey, Ez through the ground level |0>, described by its 4x4 density
 * matrix (the paper writes it as a real su(4) vector), with population decay
 * time T1, dephasing time T2 and an incoherent pump.  Normalised units
 * (hbar = 1 in units of hbar c / a, field unit E0 = hbar c / (mu a)):
 *   H = w0 (|1><1| + |2><2| + |3><3|) - sum_k E_k (|0><k| + |k><0|)
 *   d rho/dt = -i [H, rho] + relaxation,
 *   relaxation: d rho_kk/dt = -rho_kk / T1 + (pump / 3) rho_00   (k = 1..3)
 *               d rho_00/dt = sum_k rho_kk / T1 - pump rho_00
 *               d rho_ab/dt = -rho_ab / T2                       (a != b)
 *   P_k = 2 kappa Re rho_0k,  kappa = N mu^2 a / (eps0 hbar c).
 *
 * One step of the matter over dt driven by a field E (the field at the middle
 * of the step) is the symmetric splitting
 *   S(rho; E) = R(dt/2) C(E) R(dt/2) rho,
 * R the exact flow of the relaxation equations, C the Cayley (Crank-Nicolson)
 * propagator rho -> V rho V^+, V = (I + i (dt/2) H')^{-1} (I - i (dt/2) H'),
 * with H' = H at the prewarped frequency w' = (2/dt) tan(w0 dt / 2), which makes
 * the free precession of a coherence exactly exp(i w0 dt) per step.
 */
#ifndef ORC_BLOCH_REF_H
#define ORC_BLOCH_REF_H
#include <complex.h>
#include "oracle.h"

typedef double complex orc_z;

typedef struct {
  double w0;      /* transition angular frequency 2 pi f_a (c/a units) */
  double wp;      /* prewarped (2/dt) tan(w0 dt/2) */
  double kappa;   /* P_k = 2 kappa Re rho_0k */
  double g1;      /* 1/T1 (normalised) */
  double g2;      /* 1/T2 */
  double gp;      /* pump rate */
  double noise;   /* sigma_N / sqrt(dt dx^3) */
} orc_bloch_c;

/* Constants of material m at time step dt; -1 for an invalid material. */
int orc_bloch_setup(const orc_material* m, double dt, double dx, double a_meters, orc_bloch_c* c);
/* rho <- R(tau) rho */
void orc_bloch_relax(const orc_bloch_c* c, double tau, orc_z r[4][4]);
/* rho <- V rho V^+ over dt with field E */
void orc_bloch_coherent(const orc_bloch_c* c, double dt, const double E[3], orc_z r[4][4]);
/* out = S(in; E) over dt */
void orc_bloch_step(const orc_bloch_c* c, double dt, const double E[3], orc_z in[4][4], orc_z out[4][4]);

#endif
