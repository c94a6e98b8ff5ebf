/*
 * libfdtd — MI355X (gfx950) Yee-FDTD stepper for gain-filled disordered
 * inverted opals.  C ABI: plain pointers, sizes and status codes.
 *
 * Method (C. Conti and A. Fratalocchi, arXiv:0802.3775):
 *   - Yee leapfrog FDTD with absorbing walls and an inverted-opal index
 *     profile: section "Sample and numerical approach".
 *   - Disorder r = r0 (1 + gamma xi), xi uniform in [-1/2, 1/2]: same section.
 *   - Pumped gain medium in the spheres with a stochastic spontaneous-emission
 *     source: same section and the lasing section ("3+1D simulation of lasing").
 *   - Transmitted power T(t), the Poynting flux through the output plane summed
 *     over that plane: section "Dynamical diffusion and localization".
 * Gain media: a Lorentz polarization driven by four-level rate equations, or
 * the paper's density-matrix (su(4)) model of a ground level coupled to three
 * degenerate upper levels (fdtd_material, gain = 2).
 *
 * Units: c = eps0 = mu0 = 1; lengths in a (cubic lattice constant), time in
 * a/c, frequency in c/a.  dx = 1/res, dt = courant * dx.  SI enters only through
 * the gain parameters, converted with a_meters.
 *
 * Layout: every per-cell array is [nz][ny][nx], x fastest, FP32 fields.  Yee
 * positions in units of dx: Ex (i+1/2,j,k) Ey (i,j+1/2,k) Ez (i,j,k+1/2)
 * Hx (i,j+1/2,k+1/2) Hy (i+1/2,j,k+1/2) Hz (i+1/2,j+1/2,k).  Voxel (i,j,k) owns
 * Ex, Ey, Ez at index (i,j,k): its material index sets their permittivity and
 * gain.  After n steps, E holds E^n and H holds H^{n-1/2}.
 *
 * Ownership: the library owns host metadata and the opaque handles.  Device
 * memory is owned by the caller: one arena per plan, at least
 * fdtd_required_bytes() bytes, 256-byte aligned, alive until the plan is
 * destroyed; the library never allocates device memory on the stepping path.
 * Host buffers passed in or out are the caller's and are not retained.
 *
 * Streams: device work is ordered on the caller's stream (a hipStream_t passed
 * as void*; NULL is the null stream).  fdtd_read_* and fdtd_write_* synchronize
 * that stream before returning.  A plan is not thread-safe; distinct plans are
 * independent.
 *
 * Errors: no exception crosses the ABI.  Every int-returning call returns
 * FDTD_OK (0) or a negative FDTD_E* code and records a message retrievable with
 * fdtd_last_error() (thread-local).
 */
#ifndef FDTD_H
#define FDTD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDTD_OK 0
#define FDTD_EINVAL (-1)       /* bad argument or configuration */
#define FDTD_ENOMEM (-2)       /* arena too small / host allocation failed */
#define FDTD_EHIP (-3)         /* a HIP runtime call failed */
#define FDTD_ESTATE (-4)       /* call not allowed in the plan's current state */
#define FDTD_EUNSTABLE (-5)    /* courant >= 1/sqrt(3) or an unstable oscillator */
#define FDTD_EUNSUPPORTED (-6) /* valid request outside what the library implements */

#define FDTD_MAX_MATERIALS 16
#define FDTD_MAX_SOURCES 4
#define FDTD_MAX_PROBES 16
#define FDTD_MAX_FLUX 4

enum { FDTD_BC_PERIODIC = 0, FDTD_BC_PEC = 1 };
enum { FDTD_SRC_DIPOLE = 0, FDTD_SRC_PLANE = 1, FDTD_SRC_BEAM = 2 };
enum { FDTD_WIDTH_FWHM_POWER = 0, FDTD_WIDTH_FWHM_INTENSITY = 1, FDTD_WIDTH_SIGMA_T = 2 };
enum { FDTD_DISORDER_NONE = 0, FDTD_DISORDER_UNIFORM_RADIUS = 1, FDTD_DISORDER_GAUSS_JITTER = 2 };

enum { FDTD_STORES_AUTO = 0, FDTD_STORES_ORDINARY = 1, FDTD_STORES_NONTEMPORAL = 2 };

typedef struct fdtd_plan fdtd_plan;
typedef struct fdtd_batch fdtd_batch;

/* Grid (paper, "Sample and numerical approach": the Yee grid of the FDTD code,
   a 6 um box of 200^3 cells with absorbing walls).  bc[d]: FDTD_BC_PERIODIC or
   FDTD_BC_PEC (PEC walls at both ends of axis
   d, optionally lined with pml_lo[d] / pml_hi[d] CPML layers).  CPML grading:
   sigma = sigma_max (rho/d)^m, kappa = 1 + (kappa_max - 1)(rho/d)^m,
   alpha = alpha_max (1 - rho/d); sigma_max <= 0 selects 0.8 (m + 1) / dx.
   seed / realization key the counter-based generator (geometry and noise). */
typedef struct {
  int32_t nx, ny, nz;
  int32_t bc[3];
  int32_t pml_lo[3], pml_hi[3];
  double cpml_m, cpml_sigma_max, cpml_kappa_max, cpml_alpha_max;
  int32_t res;        /* cells per lattice constant a */
  double courant;     /* dt / dx, must be < 1/sqrt(3) */
  double a_meters;    /* lattice constant in metres */
  uint32_t seed, realization;
} fdtd_grid_desc;

/* Material (paper, "Sample and numerical approach": the opal's eps_r = 12, the
   dye of index 1.3 in the spheres, its four-level Maxwell-Bloch model with T1,
   T2 and the noise source; "3+1D simulation of lasing": the pumped medium).
   eps: relative permittivity (host permittivity of a gain medium).
   gain = 1: four-level medium with total density n_total (m^-3), lifetimes
   tau32, tau21, tau10 (s), pump rate 0->3 (s^-1), Lorentz transition f_a and
   FWHM linewidth df_a (c/a), noise amplitude, initial fractions n_init[0..3].
   gain = 2: the paper's density-matrix medium (section "Sample and numerical
   approach": a ground level 0 and three degenerate upper levels 1..3 coupled to
   Ex, Ey, Ez): density n_total, transition f_a (c/a), population decay time t1
   and dephasing time t2 (s), pump rate (s^-1, 0 -> each upper level at pump/3),
   transition dipole (C m; <= 0 selects the radiative value for which t1 is the
   spontaneous lifetime in a host of index sqrt(eps)), noise amplitude (a
   current sigma_N sqrt(rho_cc) g / sqrt(dt dx^3) on E_c), initial populations
   n_init (no coherences).  Field unit hbar c / (dipole a); P_c = 2 kappa
   Re rho_0c with kappa = n_total dipole^2 a / (eps0 hbar c).  Density-matrix
   state per gain cell: 15 reals (three populations, the three ground-upper and
   three upper-upper complex coherences), the trace fixed at 1.  The gain
   materials of one plan, and of the gain members of one batch, must share one
   model (FDTD_EUNSUPPORTED otherwise). */
typedef struct {
  double eps;
  int32_t gain;
  double n_total, tau32, tau21, tau10, pump, f_a, df_a, noise;
  double n_init[4];
  double t1, t2, dipole;
} fdtd_material;

/* Source (paper, "Wide-band excitation and gap filling": the single-cycle
   linearly polarised TEM00 pulse of 2 um waist launched along [100];
   "Dynamical diffusion and localization": the 100 fs Gaussian pulse).
   s(t) = amp sin(2 pi f0 (t - t0)) exp(-(t - t0)^2 / (2 sigma_t^2)),
   t0 = delay * sigma_t.  Width: FWHM of the power spectrum (c/a), FWHM of the
   intensity envelope (a/c), or sigma_t (a/c).  DIPOLE: current s/dx^3 on E_comp
   of cell (i,j,k).  PLANE: sheet current s on E_comp over the whole z = k plane.
   BEAM (the paper's linearly polarised TEM00 beam at its waist, launched along
   z): the PLANE sheet weighted by exp(-((x - x0)^2 + (y - y0)^2) / waist^2), with
   x, y the driven component's own Yee position (Ex at ((i + 1/2) dx, j dx), Ey at
   (i dx, (j + 1/2) dx), Ez at (i dx, j dx)) and x0, y0, waist in units of a;
   waist > 0.  x0, y0, waist are ignored by the other kinds. */
typedef struct {
  int32_t kind, comp, i, j, k;
  double f0;
  int32_t width_kind;
  double width, delay, amp;
  double x0, y0, waist;
} fdtd_source_desc;

/* Inverted opal (paper, "Sample and numerical approach": air spheres of radius
   r0 = a/(2 sqrt 2) at the fcc sites of the cubic lattice, disorder r = r0 (1 +
   gamma xi) with xi uniform in [-1/2, 1/2]).  cells[3] cubic fcc cells starting
   at grid index origin[3];
   air-sphere radius r0 (units of a); disorder with strength gamma (uniform
   radius) or delta/a (Gaussian jitter of radii and centres, truncated at
   4 delta).  Voxels inside any sphere get mat_void, the rest of the crystal
   mat_bg, everything outside the crystal mat_out.  A periodic axis must be
   spanned exactly by the crystal. */
typedef struct {
  int32_t cells[3], origin[3];
  double r0;
  int32_t disorder;
  double strength;
  int32_t mat_bg, mat_void, mat_out;
} fdtd_opal_desc;

/* Launch tuning (per plan; an implementation choice the paper does not touch:
   results do not depend on it).  block: threads per workgroup, one (i,j) column per
   thread (64..256, multiple of 64); tile_x: tile width along x (16, 32 or 64;
   the tile is tile_x x block/tile_x columns, and its one-cell halo ring,
   2 (tile_x + 2) + 2 block/tile_x cells, must not exceed block: 16 with any
   block, 32 with 128 or 256, 64 with 256); zchunk: z-planes per tile (>= 1);
   graph_steps: steps captured per hipGraph (0: no graph); max_blocks: upper
   bound on resident workgroups for the tile loop (0: one per tile).
   merge: 0 one launch per tile class; 1 tiles without CPML run with the z-CPML
   kernel of the same gain flag (one launch for both); 2 every tile runs with the
   plan's most general kernel (one launch per step).  parallel: 1 makes the
   launches of a step parallel branches of the captured graph, 0 keeps them in
   stream order.  stores: FDTD_STORES_AUTO (non-temporal field stores for a plan
   whose step state exceeds four times the 256 MB Infinity Cache, ordinary ones
   otherwise and in batches), FDTD_STORES_ORDINARY or FDTD_STORES_NONTEMPORAL.
   cache_mb (batches only; >= 0): members are stepped in groups of consecutive
   members whose step state together is at most cache_mb MB, each group for all
   the steps of a call (or of a captured graph) before the next, so that a group
   that fits the Infinity Cache is read from there; 0 steps every member every
   step.  Results do not depend on any of these. */
typedef struct {
  int32_t block, zchunk, graph_steps, max_blocks, tile_x, merge, parallel, stores, cache_mb;
} fdtd_tuning;

/* Message of the last failed call on this thread; library version string. */
const char* fdtd_last_error(void);
const char* fdtd_version(void);

/* Create a plan (host only): the Yee grid of "Sample and numerical approach".
   Checks sizes, boundaries and the Courant limit (FDTD_EUNSTABLE). *out owned by
   the caller until fdtd_plan_destroy, which also releases the plan's graphs. */
int fdtd_plan_create(const fdtd_grid_desc* g, fdtd_plan** out);
void fdtd_plan_destroy(fdtd_plan* p);

/* Material table (n <= FDTD_MAX_MATERIALS; "Sample and numerical approach").
   Coefficients are built in FP64 and rounded once to FP32.  FDTD_EINVAL for bad
   parameters, FDTD_EUNSUPPORTED for two gain models in one plan. */
int fdtd_set_materials(fdtd_plan* p, const fdtd_material* tab, int32_t n);

/* Build the opal ("Sample and numerical approach": the inverted opal and its
   random-number disorder): the sphere list on the host (FP64, Philox key (seed,
   realization), counter (site id, 0, 0, 0)) quantized to integers, then the
   integer-exact voxelization on the device at bind.  Site id = h + (2nx+1)(k +
   (2ny+1) l) for fcc sites (h, k, l)/2.  Alternatively give the map directly. */
int fdtd_build_opal(fdtd_plan* p, const fdtd_opal_desc* d);
int fdtd_set_material_map(fdtd_plan* p, const uint8_t* host_map);
/* Quantized spheres of the opal (same passage): rows (site id, Cx, Cy, Cz, rho)
   in units of a/(2 res 2^16) relative to the crystal origin.  out may be NULL to
   query n; out holds 5 n int64 (caller-owned). */
int fdtd_get_spheres(const fdtd_plan* p, int64_t* out, int64_t* n);
/* Voxelized material map (after bind), [nz][ny][nx] bytes into caller memory:
   the index profile of the Fig. 1 inset.  Synchronizes the stream. */
int fdtd_get_material_map(fdtd_plan* p, uint8_t* host_map, void* stream);

/* Add a source (the excitations of "Wide-band excitation and gap filling" and
   "Dynamical diffusion and localization", or a point dipole); *id (may be NULL)
   its index.  At most FDTD_MAX_SOURCES; FDTD_EINVAL outside the grid. */
int fdtd_add_source(fdtd_plan* p, const fdtd_source_desc* s, int32_t* id);
/* Probe ("Wide-band excitation and gap filling": the field retrieved at a low
   symmetry point inside the sample) of component comp (0..5 = Ex Ey Ez Hx Hy Hz)
   at (i,j,k), recorded after every step (E^{n+1}, H^{n+1/2}). */
int fdtd_add_probe(fdtd_plan* p, int32_t comp, int32_t i, int32_t j, int32_t k, int32_t* id);
/* Flux plane ("Dynamical diffusion and localization": the transmitted power
   T(t): the Poynting flux through the output plane, summed over it) normal
   to axis (only 2, z, the launch direction; 0 and 1 give FDTD_EUNSUPPORTED) at
   index k: T(t_{n+1/2}) = sum over the plane of the time-centred S_z dx^2 every
   step, and the running DFT of Ex, Ey (time n) and the z-averaged Hx, Hy (time
   n+1/2) at nf frequencies f (c/a, copied) every decim steps, FP64
   accumulators. */
int fdtd_add_flux_plane(fdtd_plan* p, int32_t axis, int32_t k, const double* f, int32_t nf, int32_t decim,
                        int32_t* id);
/* Energy ("3+1D simulation of lasing": the stored electromagnetic energy
   density) W^n = 1/2 sum (eps |E^n|^2 + H^{n-1/2} . H^{n+1/2}) dx^3 every ke
   steps (0: off). */
int fdtd_set_energy_interval(fdtd_plan* p, int32_t ke);
/* Launch tuning (no passage of the paper; fdtd_tuning above).  Fixed at bind:
   call before fdtd_required_bytes / fdtd_bind_arena. */
int fdtd_set_tuning(fdtd_plan* p, const fdtd_tuning* t);
int fdtd_get_tuning(const fdtd_plan* p, fdtd_tuning* t);

/* Device bytes the plan needs for up to max_steps steps (layout of the arena;
   no passage of the paper: the run length of "Wide-band excitation" is 10^5
   steps). */
int fdtd_required_bytes(fdtd_plan* p, int64_t max_steps, size_t* bytes);
/* Bind the caller's device arena (no passage of the paper: device memory) dev
   (>= fdtd_required_bytes, 256-byte aligned,
   owned by the caller and alive until destroy): fixes the layout, zero-fills,
   uploads tables, voxelizes.  After this the plan's configuration is frozen.
   FDTD_ENOMEM if bytes is too small; synchronizes the stream. */
int fdtd_bind_arena(fdtd_plan* p, void* dev, size_t bytes, int64_t max_steps, void* stream);

/* Advance n leapfrog steps ("Sample and numerical approach": FDTD after
   Taflove, with the Maxwell-Bloch gain cells) on the stream, asynchronous;
   FDTD_ESTATE past max_steps, leaving the state untouched.  Step count, cell
   count and dt of the plan. */
int fdtd_step(fdtd_plan* p, int64_t n, void* stream);
int64_t fdtd_step_count(const fdtd_plan* p);
int64_t fdtd_cell_count(const fdtd_plan* p);
double fdtd_dt(const fdtd_plan* p);

/* The Yee fields ("Sample and numerical approach"): component comp (0..5) of
   the current step, nx*ny*nz floats in host
   memory (caller-owned, dense [nz][ny][nx]; on the device rows may be padded
   for alignment, which the copies undo); write sets initial conditions.
   Synchronize. */
int fdtd_read_field(fdtd_plan* p, int32_t comp, float* host, void* stream);
int fdtd_write_field(fdtd_plan* p, int32_t comp, const float* host, void* stream);
/* Probe samples (the probe of "Wide-band excitation and gap filling") 0..n-1
   (n = steps taken) into host floats (max_steps room). */
int fdtd_read_probe(fdtd_plan* p, int32_t id, float* host, int64_t* n, void* stream);
/* T(t) samples (n = steps taken, may be NULL) and the flux spectrum
   P(f) = Re sum (Ex Hy* - Ey Hx*) dx^2 (nf values, may be NULL) of flux plane id
   ("Dynamical diffusion and localization"; the spectra of Fig. 1). */
int fdtd_read_flux(fdtd_plan* p, int32_t id, double* T, double* spec, int64_t* n, void* stream);
/* Populations n0..n3 of the four-level medium ("Sample and numerical approach":
   the four-level system; the density matrix's diagonal for gain = 2), 4 * cells
   doubles, zero outside gain cells.  The device holds n1..n3 as FP32 (hi, lo)
   pairs, so that the small per-step changes of a weak pump are not rounded
   away; each level is returned as the exact sum of its pair.  n0 is not
   stored: it is 1 - (n1 + n2 + n3), so the sum of the four is 1 by
   construction. */
int fdtd_read_populations(fdtd_plan* p, double* host, void* stream);
/* Polarization P^n of the gain cells (same passage), 3 * cells floats. */
int fdtd_read_polarization(fdtd_plan* p, float* host, void* stream);
/* Density matrix ("Sample and numerical approach": the su(4) real form of the
   four-level density matrix) of a gain = 2 plan, 15 * cells floats: rho_11, rho_22, rho_33,
   Re rho_01, Re rho_02, Re rho_03, Im rho_01, Im rho_02, Im rho_03, Re rho_12,
   Re rho_13, Re rho_23, Im rho_12, Im rho_13, Im rho_23 (zero outside gain
   cells).  FDTD_ESTATE for plans without such a medium. */
int fdtd_read_density(fdtd_plan* p, float* host, void* stream);
/* Energy samples ("3+1D simulation of lasing": the stored energy) W^0, W^ke,
   ... (n returned) into host doubles. */
int fdtd_read_energy(fdtd_plan* p, double* host, int64_t* n, void* stream);

/* Batches ("Wide-band excitation and gap filling": results averaged over 10
   realizations of the disorder): bound plans that step together, one launch
   per tile class per step over all plans' tiles (uneven sizes, each plan's own
   step count).  t (may be NULL: the first member's tuning) gives the batch's
   launch settings (graph_steps, max_blocks, parallel, stores, cache_mb); its
   block and tile_x must equal every member's (their tiles were laid out at
   bind; zchunk and merge of t are not used).  Stepping a batch advances every member;
   members must stay alive.  Creation allocates the batch's launch tables on the
   device (hipMalloc; freed by destroy). */
int fdtd_batch_create(fdtd_plan* const* plans, int32_t n, const fdtd_tuning* t, fdtd_batch** out);
/* For callers that cannot allocate device memory (code under HIP graph capture,
   tight serving loops, harnesses that forbid hipMalloc): fdtd_batch_create with
   the batch's launch tables placed in a static per-GPU array of 16 MiB (held
   until the process ends) instead of a hipMalloc'd block; calls no hipMalloc or
   hipFree.  FDTD_ENOMEM if the tables need more than 16 MiB (about 300,000
   tiles of step work).  All static batches of one GPU share that array: creating
   one replaces the tables of the previous one, which from then on refuses to
   step (FDTD_ESTATE); creations that overlap on one GPU race.  Members grow into
   the same array with fdtd_batch_set_members up to the same limit. */
int fdtd_batch_create_static(fdtd_plan* const* plans, int32_t n, const fdtd_tuning* t, fdtd_batch** out);
/* Replace a batch's members (same conditions as at creation; the batch keeps
   its tuning) for continuous batching: requests join and leave between launches
   without a new batch.  The device tables are rewritten in place and grow
   (hipMalloc, once per new maximum) only when the new list needs more room; the
   batch's captured graphs are dropped.  Synchronizes the stream first, since
   launches already queued read the old tables.  A plan may belong to several
   batches, but only one of them may step it at a time. */
int fdtd_batch_set_members(fdtd_batch* b, fdtd_plan* const* plans, int32_t n, void* stream);
int fdtd_batch_step(fdtd_batch* b, int64_t n, void* stream);
void fdtd_batch_destroy(fdtd_batch* b);

/* Measurement (no passage of the paper; it prints no performance figure).
   Time n steps of the bound plan (hipEvents recorded on the stream around the
   launches; the plan's state advances).  Milliseconds in *ms. */
int fdtd_time_steps(fdtd_plan* p, int64_t n, void* stream, double* ms);
/* Same for a batch. */
int fdtd_batch_time_steps(fdtd_batch* b, int64_t n, void* stream, double* ms);

/* Autotuning (no passage of the paper: launch tuning): time ncand candidate
   tunings of plan p (bound or not; p itself is
   not touched) on scratch plans with p's description and each candidate's
   tuning, bound in turn to the caller's scratch arena (device memory, 256-byte
   aligned, bytes long): warmup untimed steps, then steps timed ones on the
   stream.  ms[q] = milliseconds per step, -1 for an invalid tuning, -2 if the
   candidate needs more than bytes.  need (may be NULL) receives the largest
   arena any candidate needs; with scratch NULL only need is computed.  Allocates
   no device memory itself. */
int fdtd_tune(const fdtd_plan* p, const fdtd_tuning* cand, int32_t ncand, int64_t warmup, int64_t steps,
              void* scratch, size_t bytes, size_t* need, double* ms, void* stream);

/* Kernels of a step (FDTD_NKERNEL entries): 0 plain tiles, 1 tiles touching
   z-CPML slabs only, 2 tiles touching x or y slabs, 3-5 the same with Lorentz
   gain cells; 6 the running-DFT update; 7-10 the passes of the density-matrix
   medium (predictor, corrector, edges, diagnostics).  cells[c] = cells covered
   by the plan's tiles of class c (c < 6), flux-plane points (6), gain cells (7,
   8), cells whose edges a gain cell shares (9), flux-plane points and probes
   (10). */
#define FDTD_NKERNEL 11
int fdtd_class_cells(const fdtd_plan* p, int64_t* cells /* FDTD_NKERNEL */);
/* Algorithmic bytes one launch of each kernel moves (FDTD_NKERNEL entries):
   49 per cell (E, H and the material index in, E and H out) + 32 per cell and
   CPML axis whose slab holds it (2 E-side psi read+write, 2 H-side psi read +
   write) + 4 per cell of a Lorentz gain tile (its gain ordinal) + 84 per
   Lorentz gain cell (P^n, P^{n-1}, populations in; P^{n+1}, populations out);
   the DFT entry is the average bytes of one call: the plane sample (24 bytes
   read, 16 written per point) and, once per 32 samples, the 4 complex FP64
   accumulators read + written per plane point and frequency plus the sample
   ring read; per density-matrix gain cell 113 (predictor: 18 state floats, the
   cell's share of E^n and A, map and list, Q*) and 197 (corrector: the state
   read and written, fields, neighbours' Q*, Q), 41 per cell whose edges a gain
   cell shares (its list entry, the sharers' Q, A in, E out, map), 32 per
   flux-plane point + 8 per probe for the diagnostics. */
int fdtd_class_bytes(const fdtd_plan* p, double* bytes /* FDTD_NKERNEL */);
/* Advance n steps without graphs, launching every kernel with a pair of hipEvents
   bound to the launch (hipExtLaunchKernelGGL start/stop: the kernel's own begin
   and end timestamps); ms[c] = summed milliseconds and launches[c] = number of
   launches of kernel c (FDTD_NKERNEL entries each, as above). */
int fdtd_time_kernels(fdtd_plan* p, int64_t n, void* stream, double* ms, int64_t* launches);
/* The same for a batch, member group after member group: ms[c] sums kernel c's
   launches over all groups, and launches[c] counts the steps in which it ran, so
   ms[c] / launches[c] is its time per batch step over all members (whose bytes
   are the sum of the members' fdtd_class_bytes). */
int fdtd_batch_time_kernels(fdtd_batch* b, int64_t n, void* stream, double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif
