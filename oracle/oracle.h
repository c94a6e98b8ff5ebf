/*
 * FP64 CPU oracle for the inverted-opal Yee / Lorentz / four-level stepper.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library, and it never reads anything the GPU
 * path produced.
 *
 * Paper: C. Conti and A. Fratalocchi, "Dynamic light diffusion, Anderson
 * localization and lasing in disordered inverted opals: 3D ab-initio
 * Maxwell-Bloch computation" (arXiv:0802.3775).
 *   - Yee FDTD with absorbing walls: section "Sample and numerical approach".
 *   - Inverted opal (air spheres at fcc sites, eps_r background, r0 = a/(2 sqrt 2)),
 *     disorder r = r0 (1 + gamma xi), xi uniform in [-1/2, 1/2]: same section.
 *   - Gain medium pumped externally, spontaneous emission as a stochastic
 *     source: same section and the lasing section.
 *   - Transmitted power T(t): the Poynting flux through the output plane,
 *     summed over that plane; section "Dynamical diffusion and localization".
 * Two gain models: a Lorentz polarization driven by four-level population
 * rate equations (gain = 1), and the paper's density-matrix model of a ground
 * level coupled to three degenerate upper levels (gain = 2, bloch_ref.h).
 *
 * Units: c = eps0 = mu0 = 1; lengths in a, time in a/c, frequency in c/a.
 * Grid pitch dx = 1/res, time step dt = courant * dx.  Arrays are [nz][ny][nx],
 * x fastest.  Yee positions (units of dx): Ex (i+1/2,j,k), Ey (i,j+1/2,k),
 * Ez (i,j,k+1/2), Hx (i,j+1/2,k+1/2), Hy (i+1/2,j,k+1/2), Hz (i+1/2,j+1/2,k).
 * Voxel (i,j,k) owns Ex, Ey, Ez at index (i,j,k): its material sets their
 * permittivity and gain.
 */
#ifndef ORC_ORACLE_H
#define ORC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXMAT 16
#define ORC_MAXPROBE 16
#define ORC_MAXSRC 4
#define ORC_MAXFLUX 4

typedef struct {
  int32_t nx, ny, nz;
  int32_t periodic[3];          /* 1: periodic axis; 0: PEC walls at both ends */
  int32_t pml_lo[3], pml_hi[3]; /* CPML layers at each end (non-periodic axes) */
  double cpml_m;                /* grading order */
  double cpml_sigma_max;        /* <= 0 selects 0.8 (m+1) / dx */
  double cpml_kappa_max;
  double cpml_alpha_max;
  int32_t res;                  /* cells per lattice constant a */
  double courant;               /* dt / dx */
  double a_meters;              /* lattice constant in metres (SI gain parameters) */
  uint32_t seed, realization;   /* Philox key */
} orc_grid;

typedef struct {
  double eps;                   /* relative permittivity (host permittivity for gain) */
  int32_t gain;                 /* 1: Lorentz + four-level rate equations; 2: density matrix */
  double n_total;               /* m^-3 */
  double tau32, tau21, tau10;   /* s (gain 1) */
  double pump;                  /* s^-1: level 0 -> 3 (gain 1); 0 -> each upper level / 3 (gain 2) */
  double f_a, df_a;             /* transition frequency and FWHM linewidth (gain 1), c/a */
  double noise;                 /* noise amplitude sigma_N */
  double n_init[4];             /* initial fractional populations n0..n3 */
  double t1, t2;                /* s: population decay and dephasing times (gain 2) */
  double dipole;                /* C m: transition dipole (gain 2); <= 0: radiative value from t1 */
} orc_material;

enum { ORC_SRC_DIPOLE = 0, ORC_SRC_PLANE = 1, ORC_SRC_BEAM = 2 };
enum { ORC_W_FWHM_POWER = 0, ORC_W_FWHM_INTENSITY = 1, ORC_W_SIGMA_T = 2 };

typedef struct {
  int32_t kind;                 /* ORC_SRC_DIPOLE, ORC_SRC_PLANE or ORC_SRC_BEAM (sheets normal to z) */
  int32_t comp;                 /* 0 Ex, 1 Ey, 2 Ez */
  int32_t i, j, k;              /* dipole cell; sheets use k only */
  double f0;                    /* carrier frequency, c/a */
  int32_t width_kind;
  double width;                 /* see width_kind */
  double delay;                 /* t0 = delay * sigma_t */
  double amp;
  /* BEAM: a sheet like PLANE whose current is weighted by the TEM00 waist
     profile exp(-((x - x0)^2 + (y - y0)^2) / waist^2), x and y (units of a)
     taken at the driven component's own Yee position (Ex at ((i + 1/2) dx, j dx),
     Ey at (i dx, (j + 1/2) dx), Ez at (i dx, j dx)) */
  double x0, y0, waist;
} orc_source;

enum { ORC_DIS_NONE = 0, ORC_DIS_UNIFORM_RADIUS = 1, ORC_DIS_GAUSS_JITTER = 2 };

typedef struct {
  int32_t cells[3];             /* cubic cells of the photonic crystal per axis */
  int32_t origin[3];            /* grid index of the crystal's low corner */
  double r0;                    /* sphere radius, units of a */
  int32_t disorder;
  double strength;              /* gamma (uniform radius) or delta/a (Gaussian jitter) */
  int32_t mat_bg, mat_void, mat_out;
} orc_opal;

typedef struct orc_sim orc_sim;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_normals4(const uint32_t ctr[4], const uint32_t key[2], double g[4]);

/* Opal geometry: sphere list and two independent voxelizations. */
int64_t orc_opal_count(const orc_grid* g, const orc_opal* o);
int orc_opal_spheres(const orc_grid* g, const orc_opal* o, int64_t* out /* n x 5 */);
int orc_voxelize_gather(const orc_grid* g, const orc_opal* o, const int64_t* sph, int64_t n,
                        uint8_t* map);
int orc_voxelize_scatter(const orc_grid* g, const orc_opal* o, const int64_t* sph, int64_t n,
                         uint8_t* map);

/* Simulation. */
orc_sim* orc_create(const orc_grid* g, const orc_material* mats, int32_t nmat, int64_t max_steps);
void orc_destroy(orc_sim* s);
int orc_set_material_map(orc_sim* s, const uint8_t* map);
int orc_add_source(orc_sim* s, const orc_source* src);
int orc_add_probe(orc_sim* s, int32_t comp, int32_t i, int32_t j, int32_t k);
int orc_add_flux_plane(orc_sim* s, int32_t k, const double* f, int32_t nf, int32_t decim);
int orc_set_energy_interval(orc_sim* s, int32_t ke);
int orc_step(orc_sim* s, int64_t n);
int64_t orc_step_count(const orc_sim* s);
int orc_get_field(const orc_sim* s, int32_t comp, double* out);   /* 0..5: Ex Ey Ez Hx Hy Hz */
int orc_set_field(orc_sim* s, int32_t comp, const double* in);
int orc_get_populations(const orc_sim* s, double* out);          /* 4 x cells, n0..n3 */
int orc_get_polarization(const orc_sim* s, double* out);         /* 3 x cells, P^n */
/* Density matrix of gain-2 cells, 15 x cells: rho_11, rho_22, rho_33,
   Re rho_01, Re rho_02, Re rho_03, Im rho_01, Im rho_02, Im rho_03,
   Re rho_12, Re rho_13, Re rho_23, Im rho_12, Im rho_13, Im rho_23 (zero elsewhere). */
int orc_get_density(const orc_sim* s, double* out);
/* Matter alone (gain-2 material m, no Maxwell): nsteps steps of the splitting
   of bloch_ref.h driven by emid (nsteps x 3); rho is 4x4 row-major (re, im)
   pairs, in/out; hist (nsteps x 32) or NULL. */
int orc_bloch_evolve(const orc_material* m, double dt, double dx, double a_meters, int64_t nsteps,
                     const double* emid, double* rho, double* hist);
/* w0, prewarped w', kappa, 1/T1, 1/T2, pump of a gain-2 material (normalised). */
int orc_bloch_constants(const orc_material* m, double dt, double dx, double a_meters, double* out6);
int64_t orc_get_probe(const orc_sim* s, int32_t id, double* out);
int64_t orc_get_flux(const orc_sim* s, int32_t id, double* T, double* spec);
int64_t orc_get_energy(const orc_sim* s, double* out);
double orc_dt(const orc_sim* s);
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
