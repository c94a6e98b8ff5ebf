/*
 * FP64 reference stepper (test infrastructure only; see oracle.h).
 *
 * One step n -> n+1, in this order:
 *   1. H^{n+1/2} = H^{n-1/2} - (dt/dx) curl E^n            (Yee; paper cites Taflove)
 *      with CFS-CPML stretching d/dw -> (1/kappa) d/dw + psi in absorbing slabs
 *      (the paper uses UPML walls; CPML is this implementation's absorber).
 *   2. noise F^n in gain cells (spontaneous emission as a stochastic source).
 *   3. Lorentz polarization, central differences in time:
 *        P^{n+1} = C1 P^n + C2 P^{n-1} + C3 (kappa' dn^n E^n + F^n),  dn = n1 - n2.
 *   4. E^{n+1} = E^n + dt/(eps dx) (curl H^{n+1/2} - dx J^{n+1/2}) - (P^{n+1}-P^n)/eps.
 *   5. four-level populations by Crank-Nicolson with the stimulated transfer
 *        u = sum_c (E_c^n + E_c^{n+1})/2 (P_c^{n+1} - P_c^n)/dt   (-u from n1, +u to n2).
 * Density-matrix gain cells (bloch_ref.h) hold their density matrix at the
 * cell centre (where the paper places the density-matrix solution, section
 * "Sample and numerical approach") and replace 2-5 by: A = E^n + dt/(eps dx) (curl H - dx J) on
 * every edge; at each gain-cell centre the average <.> of the four edges of
 * each component; and one predictor-corrector pass of the implicit midpoint
 * coupling,
 *        E^(0) = <(E^n + A)/2>,  rho* = S(rho^n; E^(0)),  Q* = P(rho*) - P(rho^n) + dt J,
 *        E*    = A - [Q*]/eps,
 *        E^(1) = <(E^n + E*)/2>, rho^{n+1} = S(rho^n; E^(1)), Q = P(rho^{n+1}) - P(rho^n) + dt J,
 *        E^{n+1} = A - [Q]/eps,
 * where [Q] on an edge is a quarter of the sum of Q over the (up to four) cells
 * that share the edge (the adjoint of the average, so sum_edges E [Q] =
 * sum_cells <E> Q), P_c(rho) = 2 kappa Re rho_0c, eps the permittivity of the
 * edge's own voxel, and J the spontaneous-emission noise current
 * sigma_N sqrt(rho_cc) g_c / sqrt(dt dx^3) at the centre.
 *   6. diagnostics: probes E^{n+1}; transmitted power T at the flux plane
 *      (paper, section "Dynamical diffusion and localization": the Poynting
 *      flux summed over the plane); running DFT of the plane fields; energy.
 * Where the paper leaves a point open (the gain model, coupling constant,
 * noise form, absorber parameters, source shapes) the choice made is the one
 * stated at the function that implements it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"
#include "bloch_ref.h"

#define PI 3.141592653589793238462643383279502884
#define C_LIGHT 299792458.0

typedef struct {
  int kf;
  int nf, decim;
  double* f;
  double* T;     /* [max_steps] */
  double* acc;   /* [4][nf][npts][2]: Ex-hat, Ey-hat, Hx-hat, Hy-hat */
  double* ex0;   /* E^n copy of the plane, x and y */
  double* ey0;
} flux_t;

struct orc_sim {
  orc_grid g;
  int nmat;
  orc_material mat[ORC_MAXMAT];
  double dx, dt;
  int64_t nx, ny, nz, ncell;
  double* E[3];
  double* H[3];
  double* Hprev[3]; /* H^{n-1/2} kept for the energy diagnostic */
  uint8_t* map;
  /* CPML: per axis 1-D coefficients at E positions (integer) and H positions (half) */
  int has_pml[3];
  double *kE[3], *bE[3], *cE[3], *kH[3], *bH[3], *cH[3];
  double* psiE[3][3]; /* [component][derivative axis] */
  double* psiH[3][3];
  /* gain */
  int has_gain;
  double* P[3];
  double* Pold[3];
  double* N[4];
  double C1[ORC_MAXMAT], C2[ORC_MAXMAT], C3[ORC_MAXMAT], kap[ORC_MAXMAT];
  double M[ORC_MAXMAT][4][4], B[ORC_MAXMAT][4][4];
  /* density-matrix gain */
  int has_bloch;
  orc_bloch_c bc[ORC_MAXMAT];
  orc_z* rho;       /* [ncell][4][4], zero outside gain-2 cells */
  double* Eo[3];    /* E^n of every edge during a density-matrix step */
  double* Es[3];    /* E* of every edge (predictor field) */
  double* Qd[3];    /* per cell: polarization increment of the predictor / corrector + dt J */
  double* Jd[3];    /* per cell: dt J, the noise current's polarization increment */
  double* Pd[3];    /* per cell: P(rho^n) */
  /* sources */
  int nsrc;
  orc_source src[ORC_MAXSRC];
  double sig_t[ORC_MAXSRC], t0[ORC_MAXSRC];
  /* probes */
  int nprobe;
  int pc[ORC_MAXPROBE];
  int64_t pidx[ORC_MAXPROBE];
  double* plog[ORC_MAXPROBE];
  /* flux planes */
  int nflux;
  flux_t flux[ORC_MAXFLUX];
  /* energy */
  int ke;
  double* elog;
  double* wplane; /* per-plane partial sums */
  int64_t step, max_steps;
};

/* ---------------------------------------------------------------- helpers */

static int64_t idx3(const orc_sim* s, int64_t i, int64_t j, int64_t k) {
  return (k * s->ny + j) * s->nx + i;
}

/* Field value at (i,j,k) with periodic wrap; beyond a PEC wall the tangential
   E that is ever read there is zero, so out-of-range reads return 0. */
static double at(const orc_sim* s, const double* F, int64_t i, int64_t j, int64_t k) {
  const int64_t n[3] = {s->nx, s->ny, s->nz};
  int64_t p[3] = {i, j, k};
  for (int d = 0; d < 3; ++d) {
    if (p[d] < 0 || p[d] >= n[d]) {
      if (!s->g.periodic[d]) return 0.0;
      p[d] = ((p[d] % n[d]) + n[d]) % n[d];
    }
  }
  return F[idx3(s, p[0], p[1], p[2])];
}

static double* zalloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

/* CFS-CPML grading (Roden and Gedney): depth rho from the interface, d = slab width. */
static void cpml_coeff(const orc_sim* s, int axis, double pos, double* kinv, double* b, double* c) {
  const int64_t n[3] = {s->nx, s->ny, s->nz};
  const double nlo = s->g.pml_lo[axis], nhi = s->g.pml_hi[axis];
  double rho = 0.0, d = 1.0;
  if (nlo > 0 && pos < nlo) { rho = nlo - pos; d = nlo; }
  else if (nhi > 0 && pos > (double)n[axis] - nhi) { rho = pos - ((double)n[axis] - nhi); d = nhi; }
  const double m = s->g.cpml_m;
  const double smax = s->g.cpml_sigma_max > 0.0 ? s->g.cpml_sigma_max : 0.8 * (m + 1.0) / s->dx;
  const double x = rho / d;
  const double sigma = smax * pow(x, m);
  const double kappa = 1.0 + (s->g.cpml_kappa_max - 1.0) * pow(x, m);
  const double alpha = s->g.cpml_alpha_max * (1.0 - x);
  *kinv = 1.0 / kappa;
  *b = exp(-(sigma / kappa + alpha) * s->dt);
  *c = sigma > 0.0 ? sigma * (*b - 1.0) / (sigma * kappa + kappa * kappa * alpha) : 0.0;
}

static int in_slab(const orc_sim* s, int axis, int64_t p) {
  const int64_t n[3] = {s->nx, s->ny, s->nz};
  return s->has_pml[axis] && (p < s->g.pml_lo[axis] || p >= n[axis] - s->g.pml_hi[axis]);
}

/* 4x4 inverse by Gauss-Jordan with partial pivoting. */
static int inv4(double A[4][4], double R[4][4]) {
  double W[4][8];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 8; ++c) W[r][c] = c < 4 ? A[r][c] : (c - 4 == r ? 1.0 : 0.0);
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabs(W[r][c]) > fabs(W[piv][c])) piv = r;
    if (W[piv][c] == 0.0) return -1;
    for (int q = 0; q < 8; ++q) { double t = W[c][q]; W[c][q] = W[piv][q]; W[piv][q] = t; }
    double inv = 1.0 / W[c][c];
    for (int q = 0; q < 8; ++q) W[c][q] *= inv;
    for (int r = 0; r < 4; ++r) {
      if (r == c) continue;
      double f = W[r][c];
      for (int q = 0; q < 8; ++q) W[r][q] -= f * W[c][q];
    }
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) R[r][c] = W[r][c + 4];
  return 0;
}

/* Gain constants for material m (normalised units). */
static int setup_gain(orc_sim* s, int m) {
  const orc_material* mt = &s->mat[m];
  const double dt = s->dt, a = s->g.a_meters;
  const double w = 2.0 * PI * mt->f_a;
  const double dw = 2.0 * PI * mt->df_a;
  const double den = 1.0 + dw * dt / 2.0;
  s->C1[m] = (2.0 - w * w * dt * dt) / den;
  s->C2[m] = (dw * dt / 2.0 - 1.0) / den;
  s->C3[m] = dt * dt / den;
  /* classical-oscillator coupling from the spontaneous lifetime tau21 */
  s->kap[m] = 6.0 * PI * mt->n_total * a * a * a * a / (w * w * C_LIGHT * mt->tau21);
  /* rate matrix dN/dt = A N: pump 0->3, decays 3->2, 2->1, 1->0 (normalised time) */
  const double t_unit = a / C_LIGHT;
  const double pr = mt->pump * t_unit;
  const double r32 = t_unit / mt->tau32, r21 = t_unit / mt->tau21, r10 = t_unit / mt->tau10;
  double A[4][4] = {{0}};
  A[3][0] += pr;  A[0][0] -= pr;
  A[2][3] += r32; A[3][3] -= r32;
  A[1][2] += r21; A[2][2] -= r21;
  A[0][1] += r10; A[1][1] -= r10;
  double L[4][4], Rm[4][4], Li[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      L[r][c] = (r == c ? 1.0 : 0.0) - 0.5 * dt * A[r][c];
      Rm[r][c] = (r == c ? 1.0 : 0.0) + 0.5 * dt * A[r][c];
    }
  if (inv4(L, Li)) return -1;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double acc = 0.0;
      for (int q = 0; q < 4; ++q) acc += Li[r][q] * Rm[q][c];
      s->M[m][r][c] = acc;
      s->B[m][r][c] = dt * Li[r][c];
    }
  return 0;
}

/* --------------------------------------------------------------- lifecycle */

orc_sim* orc_create(const orc_grid* g, const orc_material* mats, int32_t nmat, int64_t max_steps) {
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->res < 1 || nmat < 1 || nmat > ORC_MAXMAT) return NULL;
  if (!(g->courant > 0.0) || g->courant >= 1.0 / sqrt(3.0)) return NULL;
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  s->g = *g;
  s->nmat = nmat;
  memcpy(s->mat, mats, sizeof(orc_material) * (size_t)nmat);
  s->dx = 1.0 / (double)g->res;
  s->dt = g->courant * s->dx;
  s->nx = g->nx; s->ny = g->ny; s->nz = g->nz;
  s->ncell = s->nx * s->ny * s->nz;
  s->max_steps = max_steps;
  for (int c = 0; c < 3; ++c) {
    s->E[c] = zalloc(s->ncell);
    s->H[c] = zalloc(s->ncell);
    s->Hprev[c] = zalloc(s->ncell);
  }
  s->map = (uint8_t*)calloc((size_t)s->ncell, 1);
  const int64_t n[3] = {s->nx, s->ny, s->nz};
  for (int w = 0; w < 3; ++w) {
    s->has_pml[w] = !g->periodic[w] && (g->pml_lo[w] > 0 || g->pml_hi[w] > 0);
    if (!s->has_pml[w]) continue;
    s->kE[w] = zalloc(n[w]); s->bE[w] = zalloc(n[w]); s->cE[w] = zalloc(n[w]);
    s->kH[w] = zalloc(n[w]); s->bH[w] = zalloc(n[w]); s->cH[w] = zalloc(n[w]);
    for (int64_t p = 0; p < n[w]; ++p) {
      cpml_coeff(s, w, (double)p, &s->kE[w][p], &s->bE[w][p], &s->cE[w][p]);
      cpml_coeff(s, w, (double)p + 0.5, &s->kH[w][p], &s->bH[w][p], &s->cH[w][p]);
    }
    for (int c = 0; c < 3; ++c) {
      if (c == w) continue;
      s->psiE[c][w] = zalloc(s->ncell);
      s->psiH[c][w] = zalloc(s->ncell);
    }
  }
  s->has_gain = 0;
  s->has_bloch = 0;
  for (int m = 0; m < nmat; ++m) {
    if (mats[m].gain == 1) {
      s->has_gain = 1;
      if (setup_gain(s, m)) { orc_destroy(s); return NULL; }
    } else if (mats[m].gain == 2) {
      s->has_bloch = 1;
      if (orc_bloch_setup(&mats[m], s->dt, s->dx, g->a_meters, &s->bc[m])) { orc_destroy(s); return NULL; }
    } else if (mats[m].gain != 0) {
      orc_destroy(s);
      return NULL;
    }
  }
  if (s->has_bloch) {
    s->rho = (orc_z*)calloc((size_t)s->ncell * 16, sizeof(orc_z));
    for (int c = 0; c < 3; ++c) {
      s->Eo[c] = zalloc(s->ncell);
      s->Es[c] = zalloc(s->ncell);
      s->Qd[c] = zalloc(s->ncell);
      s->Jd[c] = zalloc(s->ncell);
      s->Pd[c] = zalloc(s->ncell);
    }
  }
  if (s->has_gain) {
    for (int c = 0; c < 3; ++c) { s->P[c] = zalloc(s->ncell); s->Pold[c] = zalloc(s->ncell); }
    for (int q = 0; q < 4; ++q) s->N[q] = zalloc(s->ncell);
  }
  s->wplane = zalloc(s->nz);
  return s;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  for (int c = 0; c < 3; ++c) {
    free(s->E[c]); free(s->H[c]); free(s->Hprev[c]);
    free(s->P[c]); free(s->Pold[c]);
    for (int w = 0; w < 3; ++w) { free(s->psiE[c][w]); free(s->psiH[c][w]); }
    free(s->Eo[c]); free(s->Es[c]); free(s->Qd[c]); free(s->Jd[c]); free(s->Pd[c]);
    free(s->kE[c]); free(s->bE[c]); free(s->cE[c]);
    free(s->kH[c]); free(s->bH[c]); free(s->cH[c]);
  }
  for (int q = 0; q < 4; ++q) free(s->N[q]);
  free(s->rho);
  for (int p = 0; p < s->nprobe; ++p) free(s->plog[p]);
  for (int f = 0; f < s->nflux; ++f) {
    free(s->flux[f].f); free(s->flux[f].T); free(s->flux[f].acc);
    free(s->flux[f].ex0); free(s->flux[f].ey0);
  }
  free(s->elog); free(s->wplane); free(s->map);
  free(s);
}

int orc_set_material_map(orc_sim* s, const uint8_t* map) {
  for (int64_t q = 0; q < s->ncell; ++q)
    if (map[q] >= s->nmat) return -1;
  memcpy(s->map, map, (size_t)s->ncell);
  if (s->has_gain) {
    /* initial populations from each cell's material; non-gain cells hold none */
    for (int64_t q = 0; q < s->ncell; ++q) {
      const orc_material* mt = &s->mat[map[q]];
      for (int l = 0; l < 4; ++l) s->N[l][q] = mt->gain == 1 ? mt->n_init[l] : 0.0;
    }
  }
  if (s->has_bloch) {
    /* rho = diag(n_init) in gain-2 cells, zero elsewhere */
    for (int64_t q = 0; q < s->ncell; ++q) {
      const orc_material* mt = &s->mat[map[q]];
      orc_z* r = s->rho + 16 * q;
      for (int a = 0; a < 16; ++a) r[a] = 0.0;
      if (mt->gain == 2)
        for (int l = 0; l < 4; ++l) r[5 * l] = mt->n_init[l];
    }
  }
  return 0;
}

int orc_add_source(orc_sim* s, const orc_source* src) {
  if (s->nsrc >= ORC_MAXSRC || src->comp < 0 || src->comp > 2) return -1;
  if (src->kind == ORC_SRC_DIPOLE) {
    if (src->i < 0 || src->i >= s->nx || src->j < 0 || src->j >= s->ny || src->k < 0 || src->k >= s->nz)
      return -1;
  } else if (src->kind == ORC_SRC_PLANE) {
    if (src->k < 0 || src->k >= s->nz) return -1;
  } else if (src->kind == ORC_SRC_BEAM) {
    if (src->k < 0 || src->k >= s->nz || !(src->waist > 0.0)) return -1;
  } else {
    return -1;
  }
  double sig;
  const double sqrt_ln2 = sqrt(log(2.0));
  if (src->width_kind == ORC_W_FWHM_POWER) {
    /* power spectrum exp(-(f-f0)^2/sigma_f^2) has FWHM 2 sigma_f sqrt(ln 2) */
    double sigma_f = src->width / (2.0 * sqrt_ln2);
    sig = 1.0 / (2.0 * PI * sigma_f);
  } else if (src->width_kind == ORC_W_FWHM_INTENSITY) {
    /* intensity envelope exp(-(t-t0)^2/sigma_t^2) has FWHM 2 sigma_t sqrt(ln 2) */
    sig = src->width / (2.0 * sqrt_ln2);
  } else if (src->width_kind == ORC_W_SIGMA_T) {
    sig = src->width;
  } else {
    return -1;
  }
  s->src[s->nsrc] = *src;
  s->sig_t[s->nsrc] = sig;
  s->t0[s->nsrc] = src->delay * sig;
  return s->nsrc++;
}

int orc_add_probe(orc_sim* s, int32_t comp, int32_t i, int32_t j, int32_t k) {
  if (s->nprobe >= ORC_MAXPROBE || comp < 0 || comp > 5) return -1;
  if (i < 0 || i >= s->nx || j < 0 || j >= s->ny || k < 0 || k >= s->nz) return -1;
  int p = s->nprobe++;
  s->pc[p] = comp;
  s->pidx[p] = idx3(s, i, j, k);
  s->plog[p] = zalloc(s->max_steps);
  return p;
}

int orc_add_flux_plane(orc_sim* s, int32_t k, const double* f, int32_t nf, int32_t decim) {
  if (s->nflux >= ORC_MAXFLUX || nf < 0 || decim < 1) return -1;
  if (k < 0 || k >= s->nz || (k == 0 && !s->g.periodic[2])) return -1;
  flux_t* fl = &s->flux[s->nflux];
  fl->kf = k;
  fl->nf = nf;
  fl->decim = decim;
  fl->f = zalloc(nf);
  memcpy(fl->f, f, sizeof(double) * (size_t)nf);
  fl->T = zalloc(s->max_steps);
  fl->acc = zalloc(4 * (int64_t)nf * s->nx * s->ny * 2);
  fl->ex0 = zalloc(s->nx * s->ny);
  fl->ey0 = zalloc(s->nx * s->ny);
  return s->nflux++;
}

int orc_set_energy_interval(orc_sim* s, int32_t ke) {
  if (ke < 1) return -1;
  s->ke = ke;
  free(s->elog);
  s->elog = zalloc(s->max_steps / ke + 1);
  return 0;
}

/* Source current at t = (n + 1/2) dt, already multiplied by dx:
   dipole J = s(t)/dx^3 (one cell), sheet K = s(t) as J = K/dx. */
static double source_dxJ(const orc_sim* s, int q, int64_t n) {
  const orc_source* src = &s->src[q];
  const double t = ((double)n + 0.5) * s->dt;
  const double tau = t - s->t0[q];
  const double sig = s->sig_t[q];
  const double w = src->amp * sin(2.0 * PI * src->f0 * tau) * exp(-tau * tau / (2.0 * sig * sig));
  return src->kind == ORC_SRC_DIPOLE ? w / (s->dx * s->dx) : w;
}

/* TEM00 waist profile of a BEAM sheet at component c of cell (i, j): the
   Gaussian exp(-r^2 / w^2) of the distance from the beam axis (x0, y0), taken
   at the component's own position in the Yee cell (units of a). */
static double beam_weight(const orc_sim* s, const orc_source* src, int c, int64_t i, int64_t j) {
  const double x = ((double)i + (c == 0 ? 0.5 : 0.0)) * s->dx;
  const double y = ((double)j + (c == 1 ? 0.5 : 0.0)) * s->dx;
  const double rx = x - src->x0, ry = y - src->y0;
  return exp(-(rx * rx + ry * ry) / (src->waist * src->waist));
}

/* ------------------------------------------------------------------- step */

static void update_H(orc_sim* s) {
  const double ch = s->dt / s->dx;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < s->nz; ++k)
    for (int64_t j = 0; j < s->ny; ++j)
      for (int64_t i = 0; i < s->nx; ++i) {
        const int64_t q = idx3(s, i, j, k);
        const int64_t p[3] = {i, j, k};
        for (int c = 0; c < 3; ++c) {
          const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
          /* (curl E)_c = d_{a1} E_{a2} - d_{a2} E_{a1}, forward differences */
          int64_t s1[3] = {i, j, k}, s2[3] = {i, j, k};
          s1[a1] += 1;
          s2[a2] += 1;
          double d1 = at(s, s->E[a2], s1[0], s1[1], s1[2]) - s->E[a2][q];
          double d2 = at(s, s->E[a1], s2[0], s2[1], s2[2]) - s->E[a1][q];
          if (in_slab(s, a1, p[a1])) {
            double* psi = &s->psiH[c][a1][q];
            *psi = s->bH[a1][p[a1]] * *psi + s->cH[a1][p[a1]] * d1;
            d1 = d1 * s->kH[a1][p[a1]] + *psi;
          }
          if (in_slab(s, a2, p[a2])) {
            double* psi = &s->psiH[c][a2][q];
            *psi = s->bH[a2][p[a2]] * *psi + s->cH[a2][p[a2]] * d2;
            d2 = d2 * s->kH[a2][p[a2]] + *psi;
          }
          s->H[c][q] -= ch * (d1 - d2);
        }
      }
}

static void update_E_and_matter(orc_sim* s, int64_t n) {
  const double dt = s->dt, dx = s->dx;
  const double noise_norm = 1.0 / sqrt(dt * dx * dx * dx);
  const uint32_t key[2] = {s->g.seed, s->g.realization};
  double dxJ[ORC_MAXSRC];
  for (int q = 0; q < s->nsrc; ++q) dxJ[q] = source_dxJ(s, q, n);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < s->nz; ++k)
    for (int64_t j = 0; j < s->ny; ++j)
      for (int64_t i = 0; i < s->nx; ++i) {
        const int64_t q = idx3(s, i, j, k);
        const int64_t p[3] = {i, j, k};
        const int m = s->map[q];
        const orc_material* mt = &s->mat[m];
        const double eps = mt->eps;
        const double cb = dt / (eps * dx);
        double Eold[3], Pnew[3] = {0, 0, 0}, Pcur[3] = {0, 0, 0}, A[3];
        int pec[3] = {0, 0, 0};
        for (int c = 0; c < 3; ++c) Eold[c] = s->E[c][q];
        /* density-matrix plans: keep E^n of every edge for the centre coupling */
        if (s->has_bloch)
          for (int c = 0; c < 3; ++c) s->Eo[c][q] = Eold[c];
        /* 2-3: noise and Lorentz polarization in gain cells */
        if (mt->gain == 1) {
          double F[3] = {0, 0, 0};
          if (mt->noise != 0.0) {
            const uint32_t ctr[4] = {(uint32_t)n, (uint32_t)q, 0u, 2u};
            double gs[4];
            orc_normals4(ctr, key, gs);
            const double n2 = s->N[2][q] > 0.0 ? s->N[2][q] : 0.0;
            for (int c = 0; c < 3; ++c) F[c] = mt->noise * sqrt(n2) * gs[c] * noise_norm;
          }
          const double dn = s->N[1][q] - s->N[2][q];
          for (int c = 0; c < 3; ++c) {
            Pcur[c] = s->P[c][q];
            Pnew[c] = s->C1[m] * Pcur[c] + s->C2[m] * s->Pold[c][q] +
                      s->C3[m] * (s->kap[m] * dn * Eold[c] + F[c]);
          }
        }
        /* 4: E update */
        for (int c = 0; c < 3; ++c) {
          const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
          /* tangential E on a PEC wall stays zero */
          if ((!s->g.periodic[a1] && p[a1] == 0) || (!s->g.periodic[a2] && p[a2] == 0)) {
            pec[c] = 1;
            A[c] = 0.0;
            continue;
          }
          /* (curl H)_c = d_{a1} H_{a2} - d_{a2} H_{a1}, backward differences */
          int64_t s1[3] = {i, j, k}, s2[3] = {i, j, k};
          s1[a1] -= 1;
          s2[a2] -= 1;
          double d1 = s->H[a2][q] - at(s, s->H[a2], s1[0], s1[1], s1[2]);
          double d2 = s->H[a1][q] - at(s, s->H[a1], s2[0], s2[1], s2[2]);
          if (in_slab(s, a1, p[a1])) {
            double* psi = &s->psiE[c][a1][q];
            *psi = s->bE[a1][p[a1]] * *psi + s->cE[a1][p[a1]] * d1;
            d1 = d1 * s->kE[a1][p[a1]] + *psi;
          }
          if (in_slab(s, a2, p[a2])) {
            double* psi = &s->psiE[c][a2][q];
            *psi = s->bE[a2][p[a2]] * *psi + s->cE[a2][p[a2]] * d2;
            d2 = d2 * s->kE[a2][p[a2]] + *psi;
          }
          double curl = d1 - d2;
          for (int rr = 0; rr < s->nsrc; ++rr) {
            const orc_source* src = &s->src[rr];
            if (src->comp != c) continue;
            if (src->kind == ORC_SRC_DIPOLE && (src->i != i || src->j != j || src->k != k)) continue;
            if (src->kind != ORC_SRC_DIPOLE && src->k != k) continue;
            curl -= src->kind == ORC_SRC_BEAM ? dxJ[rr] * beam_weight(s, src, c, i, j) : dxJ[rr];
          }
          A[c] = Eold[c] + cb * curl;
        }
        /* density-matrix plans: E holds A until the centre coupling (bloch_cells) */
        for (int c = 0; c < 3; ++c) s->E[c][q] = pec[c] ? 0.0 : A[c] - (Pnew[c] - Pcur[c]) / eps;
        /* 5: populations */
        if (mt->gain == 1) {
          double u = 0.0;
          for (int c = 0; c < 3; ++c)
            u += 0.5 * (Eold[c] + s->E[c][q]) * (Pnew[c] - Pcur[c]) / dt;
          const double sv[4] = {0.0, -u, u, 0.0};
          double Nold[4], Nnew[4];
          for (int l = 0; l < 4; ++l) Nold[l] = s->N[l][q];
          for (int r = 0; r < 4; ++r) {
            double acc = 0.0;
            for (int l = 0; l < 4; ++l) acc += s->M[m][r][l] * Nold[l] + s->B[m][r][l] * sv[l];
            Nnew[r] = acc;
          }
          for (int l = 0; l < 4; ++l) s->N[l][q] = Nnew[l];
          for (int c = 0; c < 3; ++c) {
            s->Pold[c][q] = Pcur[c];
            s->P[c][q] = Pnew[c];
          }
        }
      }
}

/* ------------------------------------------- density matrix at cell centres */

/* Wraps index p along axis d; -1 beyond a PEC wall. */
static int64_t wrap_axis(const orc_sim* s, int d, int64_t p) {
  const int64_t n[3] = {s->nx, s->ny, s->nz};
  if (p >= 0 && p < n[d]) return p;
  if (!s->g.periodic[d]) return -1;
  return ((p % n[d]) + n[d]) % n[d];
}

/* Tangential E held at zero on a PEC wall (index 0 of a non-periodic axis
   transverse to the component). */
static int pec_held(const orc_sim* s, int c, const int64_t p[3]) {
  const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
  return (!s->g.periodic[a1] && p[a1] == 0) || (!s->g.periodic[a2] && p[a2] == 0);
}

/* Average over the four edges of component c around the centre of cell p:
   the edges sit at offsets {0, 1} along the two axes transverse to c (edges
   beyond a PEC wall hold zero). */
static double centre_average(const orc_sim* s, const double* F, int c, const int64_t p[3]) {
  const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
  double acc = 0.0;
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      int64_t e[3] = {p[0], p[1], p[2]};
      e[a1] = wrap_axis(s, a1, p[a1] + u);
      e[a2] = wrap_axis(s, a2, p[a2] + v);
      if (e[a1] < 0 || e[a2] < 0) continue;
      acc += F[idx3(s, e[0], e[1], e[2])];
    }
  return 0.25 * acc;
}

/* A quarter of the sum of Q over the (up to four) cells that share edge c of
   cell p: the cells at offsets {0, -1} along the two transverse axes. */
static double edge_share(const orc_sim* s, const double* Q, int c, const int64_t p[3]) {
  const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
  double acc = 0.0;
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      int64_t e[3] = {p[0], p[1], p[2]};
      e[a1] = wrap_axis(s, a1, p[a1] - u);
      e[a2] = wrap_axis(s, a2, p[a2] - v);
      if (e[a1] < 0 || e[a2] < 0) continue;
      acc += Q[idx3(s, e[0], e[1], e[2])];
    }
  return 0.25 * acc;
}

/* One coupling stage: every density-matrix cell steps rho^n with the centre
   average of (E^n + F)/2 (F = A for the predictor, E* for the corrector) and
   stores Q = P(new rho) - P(rho^n) + dt J; the corrector keeps the new rho. */
static void bloch_stage(orc_sim* s, double* const F[3], int keep) {
  const double dt = s->dt;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < s->nz; ++k)
    for (int64_t j = 0; j < s->ny; ++j)
      for (int64_t i = 0; i < s->nx; ++i) {
        const int64_t q = idx3(s, i, j, k);
        const int m = s->map[q];
        if (s->mat[m].gain != 2) continue;
        const int64_t p[3] = {i, j, k};
        double Em[3];
        for (int c = 0; c < 3; ++c)
          Em[c] = 0.5 * (centre_average(s, s->Eo[c], c, p) + centre_average(s, F[c], c, p));
        orc_z(*r)[4] = (orc_z(*)[4])(s->rho + 16 * q);
        orc_z t[4][4];
        orc_bloch_step(&s->bc[m], dt, Em, r, t);
        for (int c = 0; c < 3; ++c)
          s->Qd[c][q] = 2.0 * s->bc[m].kappa * creal(t[0][c + 1]) - s->Pd[c][q] + s->Jd[c][q];
        if (keep) memcpy(r, t, sizeof(t));
      }
}

/* out = A - [Q]/eps on every edge not held by a PEC wall (A is in s->E). */
static void bloch_edges(orc_sim* s, double* const out[3]) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < s->nz; ++k)
    for (int64_t j = 0; j < s->ny; ++j)
      for (int64_t i = 0; i < s->nx; ++i) {
        const int64_t q = idx3(s, i, j, k);
        const int64_t p[3] = {i, j, k};
        const double eps = s->mat[s->map[q]].eps;
        for (int c = 0; c < 3; ++c)
          out[c][q] = pec_held(s, c, p) ? 0.0 : s->E[c][q] - edge_share(s, s->Qd[c], c, p) / eps;
      }
}

/* The density-matrix cells of step n, after the edge loop has left A in s->E
   and E^n in s->Eo: noise and P(rho^n) per cell, predictor, E*, corrector,
   E^{n+1}. */
static void bloch_cells(orc_sim* s, int64_t n) {
  const uint32_t key[2] = {s->g.seed, s->g.realization};
  const double dt = s->dt;
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < s->ncell; ++q) {
    const int m = s->map[q];
    for (int c = 0; c < 3; ++c) s->Jd[c][q] = s->Pd[c][q] = s->Qd[c][q] = 0.0;
    if (s->mat[m].gain != 2) continue;
    const orc_z* r = s->rho + 16 * q;
    for (int c = 0; c < 3; ++c) s->Pd[c][q] = 2.0 * s->bc[m].kappa * creal(r[c + 1]);
    if (s->mat[m].noise != 0.0) {
      const uint32_t ctr[4] = {(uint32_t)n, (uint32_t)q, 0u, 2u};
      double gs[4];
      orc_normals4(ctr, key, gs);
      for (int c = 0; c < 3; ++c) {
        const double pc = creal(r[5 * (c + 1)]) > 0.0 ? creal(r[5 * (c + 1)]) : 0.0;
        s->Jd[c][q] = dt * s->bc[m].noise * sqrt(pc) * gs[c];
      }
    }
  }
  bloch_stage(s, s->E, 0);
  bloch_edges(s, s->Es);
  bloch_stage(s, s->Es, 1);
  bloch_edges(s, s->E);
}

static double energy_now(orc_sim* s) {
  /* W^n = 1/2 sum (eps |E^n|^2 + H^{n-1/2} . H^{n+1/2}) dx^3; called after the H
     update and before the E update */
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < s->nz; ++k) {
    double acc = 0.0;
    for (int64_t j = 0; j < s->ny; ++j)
      for (int64_t i = 0; i < s->nx; ++i) {
        const int64_t q = idx3(s, i, j, k);
        const double eps = s->mat[s->map[q]].eps;
        for (int c = 0; c < 3; ++c)
          acc += eps * s->E[c][q] * s->E[c][q] + s->Hprev[c][q] * s->H[c][q];
      }
    s->wplane[k] = acc;
  }
  double w = 0.0;
  for (int64_t k = 0; k < s->nz; ++k) w += s->wplane[k];
  return 0.5 * w * s->dx * s->dx * s->dx;
}

static void flux_before(orc_sim* s) {
  for (int f = 0; f < s->nflux; ++f) {
    flux_t* fl = &s->flux[f];
    for (int64_t j = 0; j < s->ny; ++j)
      for (int64_t i = 0; i < s->nx; ++i) {
        fl->ex0[j * s->nx + i] = s->E[0][idx3(s, i, j, fl->kf)];
        fl->ey0[j * s->nx + i] = s->E[1][idx3(s, i, j, fl->kf)];
      }
  }
}

static void flux_after(orc_sim* s, int64_t n) {
  const double dx2 = s->dx * s->dx;
  const int64_t npts = s->nx * s->ny;
  for (int f = 0; f < s->nflux; ++f) {
    flux_t* fl = &s->flux[f];
    const int64_t kf = fl->kf;
    const int64_t km = kf - 1 >= 0 ? kf - 1 : s->nz - 1; /* periodic z only when kf == 0 */
    double T = 0.0;
    for (int64_t j = 0; j < s->ny; ++j)
      for (int64_t i = 0; i < s->nx; ++i) {
        const int64_t p = j * s->nx + i;
        const double ex = 0.5 * (fl->ex0[p] + s->E[0][idx3(s, i, j, kf)]);
        const double ey = 0.5 * (fl->ey0[p] + s->E[1][idx3(s, i, j, kf)]);
        const double hx = 0.5 * (s->H[0][idx3(s, i, j, km)] + s->H[0][idx3(s, i, j, kf)]);
        const double hy = 0.5 * (s->H[1][idx3(s, i, j, km)] + s->H[1][idx3(s, i, j, kf)]);
        T += ex * hy - ey * hx;
      }
    fl->T[n] = T * dx2;
    if (n % fl->decim != 0) continue;
    const double w = (double)fl->decim * s->dt;
    for (int q = 0; q < fl->nf; ++q) {
      const double phE = 2.0 * PI * fl->f[q] * (double)n * s->dt;
      const double phH = 2.0 * PI * fl->f[q] * ((double)n + 0.5) * s->dt;
      const double cE = cos(phE), sE = sin(phE), cH = cos(phH), sH = sin(phH);
      for (int64_t j = 0; j < s->ny; ++j)
        for (int64_t i = 0; i < s->nx; ++i) {
          const int64_t p = j * s->nx + i;
          const double v[4] = {
              fl->ex0[p], fl->ey0[p],
              0.5 * (s->H[0][idx3(s, i, j, km)] + s->H[0][idx3(s, i, j, kf)]),
              0.5 * (s->H[1][idx3(s, i, j, km)] + s->H[1][idx3(s, i, j, kf)])};
          for (int c = 0; c < 4; ++c) {
            double* a = fl->acc + 2 * (((int64_t)c * fl->nf + q) * npts + p);
            const double cr = c < 2 ? cE : cH, si = c < 2 ? sE : sH;
            a[0] += v[c] * cr * w;
            a[1] += v[c] * si * w;
          }
        }
    }
  }
}

int orc_step(orc_sim* s, int64_t nsteps) {
  if (s->step + nsteps > s->max_steps) return -1;
  for (int64_t it = 0; it < nsteps; ++it) {
    const int64_t n = s->step;
    const int energy_due = s->ke > 0 && n % s->ke == 0;
    flux_before(s);
    if (energy_due)
      for (int c = 0; c < 3; ++c) memcpy(s->Hprev[c], s->H[c], sizeof(double) * (size_t)s->ncell);
    update_H(s);
    if (energy_due) s->elog[n / s->ke] = energy_now(s);
    update_E_and_matter(s, n);
    if (s->has_bloch) bloch_cells(s, n);
    flux_after(s, n);
    for (int p = 0; p < s->nprobe; ++p) s->plog[p][n] = (s->pc[p] < 3 ? s->E[s->pc[p]] : s->H[s->pc[p] - 3])[s->pidx[p]];
    s->step = n + 1;
  }
  return 0;
}

/* --------------------------------------------------------------- readout */

int64_t orc_step_count(const orc_sim* s) { return s->step; }
double orc_dt(const orc_sim* s) { return s->dt; }

int orc_get_field(const orc_sim* s, int32_t comp, double* out) {
  if (comp < 0 || comp > 5) return -1;
  memcpy(out, comp < 3 ? s->E[comp] : s->H[comp - 3], sizeof(double) * (size_t)s->ncell);
  return 0;
}

int orc_set_field(orc_sim* s, int32_t comp, const double* in) {
  if (comp < 0 || comp > 5) return -1;
  memcpy(comp < 3 ? s->E[comp] : s->H[comp - 3], in, sizeof(double) * (size_t)s->ncell);
  return 0;
}

int orc_get_populations(const orc_sim* s, double* out) {
  if (!s->has_gain && !s->has_bloch) return -1;
  for (int64_t q = 0; q < s->ncell; ++q) {
    const int g = s->mat[s->map[q]].gain;
    for (int l = 0; l < 4; ++l)
      out[l * s->ncell + q] = g == 1 ? s->N[l][q] : g == 2 ? creal(s->rho[16 * q + 5 * l]) : 0.0;
  }
  return 0;
}

int orc_get_polarization(const orc_sim* s, double* out) {
  if (!s->has_gain && !s->has_bloch) return -1;
  for (int64_t q = 0; q < s->ncell; ++q) {
    const int m = s->map[q];
    const int g = s->mat[m].gain;
    for (int c = 0; c < 3; ++c)
      out[c * s->ncell + q] = g == 1 ? s->P[c][q] : g == 2 ? 2.0 * s->bc[m].kappa * creal(s->rho[16 * q + 1 + c]) : 0.0;
  }
  return 0;
}

int orc_get_density(const orc_sim* s, double* out) {
  if (!s->has_bloch) return -1;
  const int64_t nc = s->ncell;
  static const int pr[3][2] = {{1, 2}, {1, 3}, {2, 3}};
  for (int64_t q = 0; q < nc; ++q) {
    const orc_z* r = s->rho + 16 * q;
    for (int k = 0; k < 3; ++k) {
      out[k * nc + q] = creal(r[5 * (k + 1)]);
      out[(3 + k) * nc + q] = creal(r[1 + k]);
      out[(6 + k) * nc + q] = cimag(r[1 + k]);
      out[(9 + k) * nc + q] = creal(r[4 * pr[k][0] + pr[k][1]]);
      out[(12 + k) * nc + q] = cimag(r[4 * pr[k][0] + pr[k][1]]);
    }
  }
  return 0;
}

int64_t orc_get_probe(const orc_sim* s, int32_t id, double* out) {
  if (id < 0 || id >= s->nprobe) return -1;
  memcpy(out, s->plog[id], sizeof(double) * (size_t)s->step);
  return s->step;
}

int64_t orc_get_flux(const orc_sim* s, int32_t id, double* T, double* spec) {
  if (id < 0 || id >= s->nflux) return -1;
  const flux_t* fl = &s->flux[id];
  if (T) memcpy(T, fl->T, sizeof(double) * (size_t)s->step);
  if (spec) {
    const int64_t npts = s->nx * s->ny;
    for (int q = 0; q < fl->nf; ++q) {
      double acc = 0.0;
      for (int64_t p = 0; p < npts; ++p) {
        const double* ex = fl->acc + 2 * ((0 * (int64_t)fl->nf + q) * npts + p);
        const double* ey = fl->acc + 2 * ((1 * (int64_t)fl->nf + q) * npts + p);
        const double* hx = fl->acc + 2 * ((2 * (int64_t)fl->nf + q) * npts + p);
        const double* hy = fl->acc + 2 * ((3 * (int64_t)fl->nf + q) * npts + p);
        /* Re(Ex Hy* - Ey Hx*) */
        acc += (ex[0] * hy[0] + ex[1] * hy[1]) - (ey[0] * hx[0] + ey[1] * hx[1]);
      }
      spec[q] = acc * s->dx * s->dx;
    }
  }
  return s->step;
}

int64_t orc_get_energy(const orc_sim* s, double* out) {
  if (s->ke < 1) return -1;
  int64_t n = (s->step + s->ke - 1) / s->ke;
  memcpy(out, s->elog, sizeof(double) * (size_t)n);
  return n;
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
