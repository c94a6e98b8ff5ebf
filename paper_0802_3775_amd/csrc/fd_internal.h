// Internal layout shared by the host runtime and the gfx950 kernels of libfdtd.
// Not part of the ABI (include/fdtd.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FD_MAXMAT 16
#define FD_MAXSRC 4
#define FD_MAXPROBE 16
#define FD_MAXFLUX 4
#define FD_DFT_RING 32  // flux-plane samples buffered per DFT flush
#define FD_DFT_QB 8     // frequencies per DFT work unit
#define FD_DFT_PTS 64   // plane points per DFT work unit (one per lane)
#define FD_MAXBLOCK 256   // threads per workgroup upper bound (launch bounds)
#define FD_STATIC_TABLE_BYTES ((size_t)16 << 20)  // per-GPU launch tables of batches created without allocation
#define FD_MAX_DEVICES 64

// Per-material coefficients, FP32 (built in FP64 on the host, rounded once).
struct fd_mat {
  float cb;        // dt / (eps dx)
  float inv_eps;   // 1 / eps
  float eps;       // eps (energy diagnostic)
  int is_gain;
  float C1, C2;    // Lorentz ADE: P^{n+1} = C1 P^n + C2 P^{n-1} + C3 (kappa' dn E + F)
  float C3k;       // C3 * kappa'
  float C3;
  float noise;     // sigma_N / sqrt(dt dx^3)
  float inv_dt;
  float MI[3][4];  // rows 1..3 of (M - I), M the Crank-Nicolson propagator
  float Bu[3];     // rows 1..3 of (B e2 - B e1): response to the stimulated transfer u
  float pad[3];
  // density-matrix gain (ground level + three degenerate upper levels)
  float bk2;       // 2 kappa: P_c = 2 kappa Re rho_0c
  float btau;      // dt / 2
  float bwt;       // w' dt / 2 = tan(w0 dt / 2), w' the prewarped transition frequency
  float bc1r, bc1i;  // 1 / (1 + i w' dt/2)
  float brr, bri;  // (1 - i w' dt/2) / (1 + i w' dt/2)
  float bf2;       // exp(-dt / (2 T2)): coherence decay per half step
  float beinf;     // pumped equilibrium of the upper-level total
  float bg1m;      // 1 - exp(-(pump + 1/T1) dt/2)
  float bh1m;      // 1 - exp(-dt / (2 T1))
  float bpad;
};

// One realization on the device (lives in its plan's arena).
struct fd_desc {
  int nx, ny, nz, plane;       // extents; plane = px * ny
  int px;                      // row pitch: cells from (i, j, k) to (i, j+1, k) (nx, or nx padded to 32)

  int per[3];                  // periodic axis flags
  int ncell;                   // cells per array (px ny nz), the stride of per-cell planes
  float ch;                    // dt / dx
  int nmat;
  int has_gain;
  int gain_model;     // 1: Lorentz + rate equations, 2: density matrix (one model per plan)
  unsigned gainmask;  // bit m: material m is a gain medium
  int block;                   // threads per workgroup used for this plan's tiles
  long long step;              // absolute step at batch step 0 (advanced on the device)
  long long max_steps;
  const fd_mat* mats;
  const uint8_t* mat;
  float* E[2][3];              // ping-pong by step parity
  float* H[2][3];
  float* P[2][3];              // polarization ping-pong (P^n in [n&1], P^{n-1} in the other), by gain ordinal
  // Gain state, indexed by the cell's gain ordinal gidx[cell] (gain cells
  // numbered in cell order, so a wavefront's gain cells read and write one
  // contiguous run; 0 for other cells, which never use it).  Lorentz model:
  // P[2][3] and 6 planes, n1,n2,n3 high parts, then low parts.  Density matrix:
  // 18 planes, rho_11, rho_22, rho_33 high parts, low parts, then Re rho_01..03,
  // Im rho_01..03, Re rho_12, rho_13, rho_23, Im rho_12, rho_13, rho_23.
  float* pop;
  const uint32_t* gidx;
  // Density matrix (held at the cell centre): the cell of each gain ordinal, and
  // per cell the polarization increment of the predictor (dmq[0]) and of the
  // corrector (dmq[1]), 3 planes each, both including the noise current's dt J
  // (cells without gain keep the arena's zeros)
  const uint32_t* glist;
  const uint32_t* elist;  // the (padded) cells with an edge that a gain cell shares, in cell order
  float* dmq[2];
  int ngain;
  int tile_x;  // xy tile width of the plan's step tiles (the T(t) partial slots)
  uint32_t key0, key1;
  // CPML
  int pml_lo[3], pml_hi[3], pml_t[3];
  const float* prof[3];        // per axis 6 x n_axis: kE, bE, cE, kH, bH, cH
  float* psiE[3][2];           // [axis][family], updated in place
  float* psiH[2][3][2];        // [parity][axis][family]
  // sources
  int nsrc;
  int src_kind[FD_MAXSRC], src_comp[FD_MAXSRC], src_cell[FD_MAXSRC], src_k[FD_MAXSRC];
  int src_len[FD_MAXSRC];
  const float* src_tab[FD_MAXSRC];   // dx * J(t_{n+1/2}) per step
  const float* src_prof[FD_MAXSRC];  // BEAM: transverse weight per plane cell [ny][nx]
  // probes
  int nprobe;
  int probe_comp[FD_MAXPROBE], probe_cell[FD_MAXPROBE], probe_k[FD_MAXPROBE];
  float* probe_ring;           // [nprobe][max_steps]
  // flux planes
  int nflux;
  int flux_k[FD_MAXFLUX];
  int nblk;                    // xy tiles per plane
  double* flux_T[FD_MAXFLUX];  // [max_steps][nblk] partial sums (no dx^2)
  int flux_nf[FD_MAXFLUX], flux_decim[FD_MAXFLUX];
  const double* flux_f[FD_MAXFLUX];
  double* flux_acc[FD_MAXFLUX];  // [4][nf][plane][2]
  float* flux_ring[FD_MAXFLUX];   // [FD_DFT_RING][4][plane] samples not yet added to flux_acc
  const double* flux_rot[FD_MAXFLUX];  // [nf][6]: e^{i 2pi f RING decim dt}, e^{i 2pi f decim dt}, e^{i pi f dt}
  double* flux_prev[FD_MAXFLUX];  // [4][nf][plane][2] flux_acc plus pending samples (reads)
  // energy
  int ke;
  int ntiles;
  double* energy;              // [(max_steps/ke + 1)][ntiles] partial sums (no dx^3/2)
  double dt;
};

// One unit of work: the tile_x x (block / tile_x) columns starting at (i0, j0),
// marched over z-planes [k0, k1).  tidx: index among the plan's tiles; blk: index
// of the xy tile (slot of the per-step transmitted-power partial sums).
struct fd_tile {
  const fd_desc* d;
  int i0, j0, k0, k1;
  int tidx, blk;
  // sources, probes and flux planes that touch the tile (bit q = entry q)
  unsigned srcmask, pmask, fmask;
  int flags;  // FD_TILE_ZSLAB: some plane of [k0, k1) lies in a z CPML slab
};
#define FD_TILE_ZSLAB 1

// DFT work unit: FD_DFT_PTS plane points x 4 components x FD_DFT_QB frequencies.
struct fd_dft_tile {
  const fd_desc* d;
  int flux;
  int p0;
  int q0;
  int pad;
};

// Work unit of the density-matrix passes: entries [first, first + count) of one
// plan's gain ordinals (cell passes) or of its edge list elist (edge pass); for
// the diagnostics pass first = flux plane (-1: probes), count = xy tile.
struct fd_dm_unit {
  const fd_desc* d;
  int first, count;
  int pad;
};
#define FD_DM_CELLS 256   // gain cells per unit of the cell passes (one per thread)
#define FD_DM_EDGES 256   // cells per unit of the edge pass (one per thread)

// Tile classes: kernels specialised on the CPML slabs a tile touches (none, z
// only, any axis) and on gain cells being present.  class = cpml + 3 * gain.
enum {
  FD_CLASS_PLAIN = 0, FD_CLASS_PMLZ = 1, FD_CLASS_PML = 2,
  FD_CLASS_GAIN = 3, FD_CLASS_PMLZ_GAIN = 4, FD_CLASS_PML_GAIN = 5, FD_NCLASS = 6
};
// Kernels of a step as the timing and byte counts list them: the six step
// classes, the DFT, then the four density-matrix passes.
enum { FD_KERNEL_DFT = FD_NCLASS, FD_KERNEL_DM = FD_NCLASS + 1, FD_NKERNEL = FD_NCLASS + 5 };

// Launchers (kernels.hip).
// A launch's tile list split into 8 contiguous parts of about equal cost, one
// per XCD (workgroup w runs on XCD w mod 8).  count[x] = 0 parts are allowed.
struct fd_xcd {
  int start[8];
  int count[8];
};

// part == nullptr: grid-stride loop over the tiles with the plain XCD renumbering
// start / stop (optional): events that take the kernel's own begin and end timestamps
// nt: non-temporal field stores (the launch's working set exceeds the Infinity Cache)
// Gain classes run the Lorentz medium; density-matrix plans step with the
// classes without gain and add the fd_launch_dm passes.
hipError_t fd_launch_step(int cls, const fd_tile* tiles, int ntiles, int tile_x, int block, int grid,
                          int s, const fd_xcd* part, int nt, hipStream_t st, hipEvent_t start = nullptr,
                          hipEvent_t stop = nullptr);
hipError_t fd_launch_dft(const fd_dft_tile* tiles, int ntiles, int s, hipStream_t st, hipEvent_t start = nullptr,
                         hipEvent_t stop = nullptr);
hipError_t fd_launch_dft_preview(const fd_dft_tile* tiles, int ntiles, int flux, long long first, int count,
                                 hipStream_t st);
hipError_t fd_launch_advance(fd_desc* const* descs, int n, long long k, hipStream_t st);
hipError_t fd_launch_advance_one(fd_desc* d, long long k, hipStream_t st);
hipError_t fd_launch_fill(void* p, size_t bytes, hipStream_t st);
hipError_t fd_launch_voxelize(const int64_t* sites, int ex, int ey, int ez, const int* per,
                              const int* ncr, const int* origin, const int64_t* reach,
                              int res, int mat_bg, int mat_void, int mat_out,
                              int nx, int ny, int nz, int px, uint8_t* map, hipStream_t st);
// Density-matrix passes of one step (after the step kernels have left A, the
// field before the polarization change, on every edge): predictor, corrector
// (writes rho^{n+1}), edges (E^{n+1} = A - [Q]/eps), then probes and T(t).
hipError_t fd_launch_dm(const fd_dm_unit* cells, int ncells, const fd_dm_unit* edges, int nedges,
                        const fd_dm_unit* diag, int ndiag, int block, int s, hipStream_t st,
                        hipEvent_t* ev = nullptr);
// n_init_by_mat: per material 8 floats, n0..n3 as FP32 (hi[4], lo[4]) pairs
hipError_t fd_launch_init_pop(const uint8_t* map, const float* n_init_by_mat, const uint32_t* gidx, unsigned gainmask,
                              float* pop, int ncell, int nx, int px, hipStream_t st);

// Device address of this GPU's static launch-table array (FD_STATIC_TABLE_BYTES,
// 256-byte aligned), looked up once per device with that device current.
hipError_t fd_static_tables(void** ptr, int* device);
