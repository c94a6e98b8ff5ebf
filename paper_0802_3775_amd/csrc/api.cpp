// Host runtime of libfdtd: plans, coefficient tables, arena layout, tile
// tables, graph capture, batches and read-back.  The C ABI is include/fdtd.h.
//
// Method: C. Conti and A. Fratalocchi, arXiv:0802.3775 (Yee FDTD in a
// disordered inverted opal with a pumped gain medium -- a Lorentz oscillator with
// four-level rate equations, or the paper's density matrix; sections "Sample and
// numerical approach", "Dynamical diffusion and localization", lasing section).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fdtd.h"
#include "fd_internal.h"
#include "geometry.h"

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kC = 299792458.0;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kHbar = 1.054571817e-34;

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return fail(FDTD_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Flux {
  int k, nf, decim;
  std::vector<double> f;
};

struct Layout {
  size_t total = 0;
  size_t desc, mats, ninit;
  size_t E[2][3], H[2][3];
  size_t map;
  size_t P[2][3], pop, gidx;
  size_t prof[3], psiE[3][2], psiH[2][3][2];
  size_t src[FD_MAXSRC], srcprof[FD_MAXSRC];
  size_t probe;
  size_t fluxT[FD_MAXFLUX], fluxf[FD_MAXFLUX], fluxacc[FD_MAXFLUX], fluxring[FD_MAXFLUX], fluxprev[FD_MAXFLUX];
  size_t fluxrot[FD_MAXFLUX];
  size_t energy;
  size_t tiles[FD_NCLASS];
  size_t dft;
  size_t sites;
  size_t glist, elist, dmq[2], dmunits;  // density-matrix plans: gain-cell list, Q buffers, pass work units
};

struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Side streams and events that let the tile classes of one step run as
// parallel branches of a captured graph (fork after the previous step, join
// before the DFT / next step).
struct Fork {
  hipStream_t side[FD_NCLASS] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[FD_NCLASS] = {};
  ~Fork() {
    for (int c = 0; c < FD_NCLASS; ++c) {
      if (side[c]) (void)hipStreamDestroy(side[c]);
      if (join[c]) (void)hipEventDestroy(join[c]);
    }
    if (fork) (void)hipEventDestroy(fork);
  }
  int init() {
    if (fork) return FDTD_OK;
    HIPCHK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    for (int c = 0; c < FD_NCLASS; ++c) {
      HIPCHK(hipStreamCreateWithFlags(&side[c], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&join[c], hipEventDisableTiming));
    }
    return FDTD_OK;
  }
};

// Split a tile list into 8 contiguous parts of about equal cost, one per XCD;
// *grid = 8 x the longest part (the kernel's workgroup count).
fd_xcd xcd_partition(const std::vector<double>& cost, int* grid) {
  fd_xcd r{};
  double total = 0.0;
  for (double c : cost) total += c;
  size_t idx = 0;
  double cum = 0.0;
  int longest = 0;
  for (int x = 0; x < 8; ++x) {
    r.start[x] = (int)idx;
    const double target = total * (x + 1) / 8.0;
    while (idx < cost.size() && (x == 7 || cum + 0.5 * cost[idx] <= target)) {
      cum += cost[idx];
      ++idx;
    }
    r.count[x] = (int)idx - r.start[x];
    longest = std::max(longest, r.count[x]);
  }
  *grid = 8 * std::max(longest, 1);
  return r;
}

}  // namespace

struct fdtd_plan {
  fdtd_grid_desc g{};
  double dx = 0, dt = 0;
  int64_t ncell = 0;   // cells of the grid
  // Device layout: rows of px >= nx cells (row_pitch: nx rounded up to 32
  // cells, 128 bytes, where that pads by at most an eighth), nstore = px ny nz
  // cells per array; the padding cells are never written.  Host-side arrays
  // (material map, fields read and written) are dense.
  int px = 0;
  int64_t nstore = 0;
  std::vector<fdtd_material> mats;
  bool have_opal = false;
  fdtd_opal_desc opal{};
  std::vector<int64_t> spheres;  // rows of 5
  std::vector<uint8_t> host_map; // given map, or read back after bind
  std::vector<uint32_t> gidx;     // gain ordinal of each cell (0 elsewhere)
  bool map_given = false;
  std::vector<fdtd_source_desc> sources;
  std::vector<std::array<int, 4>> probes;
  std::vector<Flux> flux;
  int ke = 0;
  fdtd_tuning tune{256, 4, 64, 0, 32, 1, 0, 0};
  // bound state
  bool bound = false;
  uint8_t* arena = nullptr;
  size_t arena_bytes = 0;
  int64_t max_steps = 0;
  Layout L;
  fd_desc hdesc{};
  fd_desc* ddesc = nullptr;
  int64_t step = 0;
  int nblk = 0, ntiles = 0;
  std::vector<fd_tile> tiles[FD_NCLASS];
  std::vector<double> tcost[FD_NCLASS];  // algorithmic bytes of each tile (XCD balancing)
  fd_xcd part[FD_NCLASS] = {};
  int pgrid[FD_NCLASS] = {};
  int ntst = 0;  // non-temporal field stores: state well beyond the Infinity Cache
  fd_tile* dtiles[FD_NCLASS] = {};
  std::vector<fd_dft_tile> dft;
  fd_dft_tile* ddft = nullptr;
  int maxnf = 0;
  // density-matrix passes: work units (cells, edges, diagnostics) and their device copy
  std::vector<fd_dm_unit> dmu[3];
  fd_dm_unit* ddm = nullptr;
  int64_t dm_cells[4] = {0, 0, 0, 0};  // cells each pass covers (predictor, corrector, edges, diagnostics)
  double dm_bytes[4] = {0, 0, 0, 0};   // algorithmic bytes of one launch of each pass
  int src_len[FD_MAXSRC] = {0, 0, 0, 0};
  bool has_gain = false;
  int gm = 0;  // gain model of the plan's gain materials: 0 none, 1 Lorentz, 2 density matrix
  hipStream_t cap = nullptr;
  std::unique_ptr<Fork> fork;
  std::map<int64_t, GraphEntry> graphs;
};

// Members [m0, m1) of a batch, stepped together: their sub-ranges of the
// batch's class tile lists, DFT units and density-matrix units (all of which
// list the members in order), with the group's own XCD partitions.
struct BGroup {
  int m0 = 0, m1 = 0;
  int t0[FD_NCLASS] = {}, nt[FD_NCLASS] = {};
  fd_xcd part[FD_NCLASS] = {};
  int pgrid[FD_NCLASS] = {};
  int d0 = 0, nd = 0;
  int u0[3] = {}, nu[3] = {};
  int maxnf = 0;
};

struct fdtd_batch {
  std::vector<fdtd_plan*> plans;
  int block = 256;
  int tile_x = 32;
  int parallel = 0;
  int max_blocks = 0;
  int graph_steps = 0;
  std::vector<fd_tile> tiles[FD_NCLASS];
  int ntst = 0;
  int cache_mb = 0;  // member groups of at most this much step state (0: one group)
  std::vector<BGroup> groups;
  int gm = 1;  // gain model shared by the members with gain
  std::vector<fd_dft_tile> dft;
  int maxnf = 0;
  std::vector<fd_dm_unit> dmu[3];  // members' density-matrix pass units
  fd_dm_unit* ddm[3] = {};
  void* dmem = nullptr;  // tile tables + desc pointer list (setup-time allocation)
  size_t dcap = 0;       // bytes available at dmem
  bool owns_dmem = false;  // dmem came from hipMalloc (freed by destroy)
  int static_dev = -1;     // static batches: the GPU whose static table array holds the tables
  uint64_t static_gen = 0;  // ... and which of that GPU's static batches wrote them last
  fd_tile* dtiles[FD_NCLASS] = {};
  fd_dft_tile* ddft = nullptr;
  fd_desc** ddescs = nullptr;
  hipStream_t cap = nullptr;
  std::unique_ptr<Fork> fork;
  std::map<std::vector<int64_t>, GraphEntry> graphs;
};

namespace {

// ------------------------------------------------------------ coefficients

// Density-matrix gain (ground level 0, upper levels 1..3 coupled to Ex, Ey, Ez),
// normalised with hbar = 1 and the field unit hbar c / (mu a):
//   H = w0 sum_k |k><k| - sum_k E_k (|0><k| + |k><0|),  P_k = 2 kappa Re rho_0k,
//   kappa = N mu^2 a / (eps0 hbar c); T1 decay of each upper level to 0, T2
//   dephasing of every coherence, pump 0 -> each upper level at pump / 3.
// A step is R(dt/2) C(E) R(dt/2): R the exact relaxation flow, C the Cayley
// map rho -> V rho V^+, V = (I + i dt/2 H')^{-1} (I - i dt/2 H') with the
// prewarped w' = (2/dt) tan(w0 dt/2) (free precession exactly exp(i w0 dt)).
int build_density_material(const fdtd_plan* p, const fdtd_material& m, fd_mat& out) {
  const double dt = p->dt, a = p->g.a_meters, tu = a / kC;
  const double w0 = 2.0 * kPi * m.f_a;
  if (!(w0 * dt < kPi)) return fail(FDTD_EUNSTABLE, "transition too fast for dt (w0 dt = %g)", w0 * dt);
  double mu = m.dipole;
  if (!(mu > 0.0)) {  // radiative value: T1 is the spontaneous lifetime in a host of index sqrt(eps)
    const double ws = w0 * kC / a;
    mu = std::sqrt(3.0 * kPi * kEps0 * kHbar * kC * kC * kC / (ws * ws * ws * std::sqrt(m.eps) * m.t1));
  }
  const double kappa = m.n_total * mu * mu * a / (kEps0 * kHbar * kC);
  const double th = std::tan(0.5 * w0 * dt);  // w' dt / 2
  const double g1 = tu / m.t1, g2 = tu / m.t2, gp = m.pump * tu;
  const double den = 1.0 + th * th;
  out.bk2 = (float)(2.0 * kappa);
  out.btau = (float)(0.5 * dt);
  out.bwt = (float)th;
  out.bc1r = (float)(1.0 / den);
  out.bc1i = (float)(-th / den);
  out.brr = (float)((1.0 - th * th) / den);
  out.bri = (float)(-2.0 * th / den);
  out.bf2 = (float)std::exp(-0.5 * g2 * dt);
  out.beinf = (float)(gp + g1 > 0.0 ? gp / (gp + g1) : 0.0);
  out.bg1m = (float)(-std::expm1(-0.5 * (gp + g1) * dt));
  out.bh1m = (float)(-std::expm1(-0.5 * g1 * dt));
  // dt J per standard normal, J = sigma_N sqrt(rho_cc) g / sqrt(dt dx^3) at the cell centre
  out.noise = (float)(m.noise * dt / std::sqrt(dt * p->dx * p->dx * p->dx));
  return FDTD_OK;
}

int build_material(const fdtd_plan* p, const fdtd_material& m, fd_mat& out) {
  std::memset(&out, 0, sizeof out);
  const double dt = p->dt, dx = p->dx;
  out.cb = (float)(dt / (m.eps * dx));
  out.inv_eps = (float)(1.0 / m.eps);
  out.eps = (float)m.eps;
  out.inv_dt = (float)(1.0 / dt);
  if (!m.gain) return FDTD_OK;
  out.is_gain = 1;
  if (m.gain == 2) return build_density_material(p, m, out);
  // Lorentz ADE by central differences:
  // (P+ - 2P + P-)/dt^2 + dw (P+ - P-)/(2dt) + w^2 P = kappa' dn E + F
  const double w = 2.0 * kPi * m.f_a, dw = 2.0 * kPi * m.df_a;
  if (w * dt >= 2.0) return fail(FDTD_EUNSTABLE, "Lorentz transition too fast for dt (w dt = %g)", w * dt);
  const double den = 1.0 + 0.5 * dw * dt;
  const double c3 = dt * dt / den;
  const double a = p->g.a_meters;
  // classical-oscillator coupling from the radiative lifetime tau21, normalised units
  const double kap = 6.0 * kPi * m.n_total * a * a * a * a / (w * w * kC * m.tau21);
  out.C1 = (float)((2.0 - w * w * dt * dt) / den);
  out.C2 = (float)((0.5 * dw * dt - 1.0) / den);
  out.C3 = (float)c3;
  out.C3k = (float)(c3 * kap);
  out.noise = (float)(m.noise / std::sqrt(dt * dx * dx * dx));
  // four-level rates in units of c/a: 0 ->3 pump, 3->2, 2->1, 1->0
  const double tu = a / kC;
  const double pr = m.pump * tu, r32 = tu / m.tau32, r21 = tu / m.tau21, r10 = tu / m.tau10;
  double A[4][4] = {};
  A[0][0] = -pr; A[3][0] = pr;
  A[3][3] = -r32; A[2][3] = r32;
  A[2][2] = -r21; A[1][2] = r21;
  A[1][1] = -r10; A[0][1] = r10;
  // Crank-Nicolson: (I - dt/2 A) N+ = (I + dt/2 A) N + dt s
  double lhs[4][8];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      lhs[r][c] = (r == c ? 1.0 : 0.0) - 0.5 * dt * A[r][c];
      lhs[r][4 + c] = r == c ? 1.0 : 0.0;
    }
  for (int c = 0; c < 4; ++c) {  // Gauss-Jordan, partial pivoting
    int pv = c;
    for (int r = c + 1; r < 4; ++r)
      if (std::fabs(lhs[r][c]) > std::fabs(lhs[pv][c])) pv = r;
    if (lhs[pv][c] == 0.0) return fail(FDTD_EINVAL, "singular population system");
    if (pv != c)
      for (int q = 0; q < 8; ++q) std::swap(lhs[c][q], lhs[pv][q]);
    const double inv = 1.0 / lhs[c][c];
    for (int q = 0; q < 8; ++q) lhs[c][q] *= inv;
    for (int r = 0; r < 4; ++r) {
      if (r == c) continue;
      const double f = lhs[r][c];
      for (int q = 0; q < 8; ++q) lhs[r][q] -= f * lhs[c][q];
    }
  }
  double Minv[4][4], M[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) Minv[r][c] = lhs[r][4 + c];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double acc = 0.0;
      for (int q = 0; q < 4; ++q) acc += Minv[r][q] * ((q == c ? 1.0 : 0.0) + 0.5 * dt * A[q][c]);
      M[r][c] = acc;
    }
  for (int r = 1; r < 4; ++r) {
    for (int c = 0; c < 4; ++c) out.MI[r - 1][c] = (float)(M[r][c] - (r == c ? 1.0 : 0.0));
    out.Bu[r - 1] = (float)(dt * (Minv[r][2] - Minv[r][1]));
  }
  return FDTD_OK;
}

// CFS-CPML grading (Roden and Gedney) at position pos (in cells) along axis w.
void cpml_point(const fdtd_plan* p, int w, double pos, float& kinv, float& b, float& c) {
  const int n = w == 0 ? p->g.nx : (w == 1 ? p->g.ny : p->g.nz);
  const double lo = p->g.pml_lo[w], hi = p->g.pml_hi[w];
  double depth = 0.0, width = 1.0;
  if (lo > 0 && pos < lo) {
    depth = lo - pos;
    width = lo;
  } else if (hi > 0 && pos > n - hi) {
    depth = pos - (n - hi);
    width = hi;
  }
  const double m = p->g.cpml_m;
  const double smax = p->g.cpml_sigma_max > 0.0 ? p->g.cpml_sigma_max : 0.8 * (m + 1.0) / p->dx;
  const double x = depth / width;
  const double sig = smax * std::pow(x, m);
  const double kap = 1.0 + (p->g.cpml_kappa_max - 1.0) * std::pow(x, m);
  const double alp = p->g.cpml_alpha_max * (1.0 - x);
  const double bb = std::exp(-(sig / kap + alp) * p->dt);
  kinv = (float)(1.0 / kap);
  b = (float)bb;
  c = (float)(sig > 0.0 ? sig * (bb - 1.0) / (sig * kap + kap * kap * alp) : 0.0);
}

double source_sigma_t(const fdtd_source_desc& s) {
  const double sl = std::sqrt(std::log(2.0));
  switch (s.width_kind) {
    case FDTD_WIDTH_FWHM_POWER: return 1.0 / (2.0 * kPi * (s.width / (2.0 * sl)));
    case FDTD_WIDTH_FWHM_INTENSITY: return s.width / (2.0 * sl);
    default: return s.width;
  }
}

int axis_n(const fdtd_plan* p, int w) { return w == 0 ? p->g.nx : (w == 1 ? p->g.ny : p->g.nz); }
// Row pitch of the device arrays.  Rows padded to a multiple of 32 cells (128
// bytes) start every tile row on a cache line: unpadded rows of 200 cells
// straddle lines in three rows of four, and padding took the step of the
// paper's 200^3 boxes from 162 to 154 us (beam) and 172 to 148 us (lasing).
// But the padding's partial line at the end of every row is moved too, so a
// row is padded only when that costs at most an eighth of it: the 80-cell rows
// of the transmission slab padded to 96 moved 11% more bytes and ran 8% slower.
int row_pitch(int nx) {
  const int p = (nx + 31) / 32 * 32;
  return (nx > 32 && 8 * (p - nx) <= p) ? p : nx;
}
// Device (padded) index of host (dense) cell o.
size_t pitched(const fdtd_plan* p, size_t o) { return (o / (size_t)p->g.nx) * (size_t)p->px + o % (size_t)p->g.nx; }
// Copies between a dense host array of ncell elements of elem bytes and the
// padded device array at dev (one row of nx elements per (j, k)).
hipError_t copy_rows_to_device(const fdtd_plan* p, void* dev, const void* host, size_t elem, hipStream_t st) {
  const size_t w = elem * (size_t)p->g.nx;
  return hipMemcpy2DAsync(dev, elem * (size_t)p->px, host, w, w, (size_t)p->g.ny * p->g.nz, hipMemcpyHostToDevice, st);
}
hipError_t copy_rows_to_host(const fdtd_plan* p, void* host, const void* dev, size_t elem, hipStream_t st) {
  const size_t w = elem * (size_t)p->g.nx;
  return hipMemcpy2DAsync(host, w, dev, elem * (size_t)p->px, w, (size_t)p->g.ny * p->g.nz, hipMemcpyDeviceToHost, st);
}
int pml_t(const fdtd_plan* p, int w) {
  return p->g.bc[w] == FDTD_BC_PEC ? p->g.pml_lo[w] + p->g.pml_hi[w] : 0;
}
size_t psi_elems(const fdtd_plan* p, int w) {
  const size_t t = (size_t)pml_t(p, w);
  const size_t nx = p->g.nx, ny = p->g.ny, nz = p->g.nz;
  if (w == 2) return t * (size_t)p->px * ny;  // z slabs are whole (padded) planes
  if (w == 0) return nz * ny * t;
  return nz * t * nx;
}

int gain_model_of(const std::vector<fdtd_material>& mats) {
  for (const fdtd_material& m : mats)
    if (m.gain) return m.gain;
  return 0;
}

// Algorithmic bytes of one gain cell per step beyond the linear 49: Lorentz
// P^n, P^{n-1}, populations in and P^{n+1}, populations out (84); density
// matrix 18 floats in and out (144).

// Bytes a step streams through: both field buffers, the material map, the psi
// slabs and the gain arrays.  Above four times the Infinity Cache (256 MB on
// MI355X) the field stores go out non-temporal; between one and four times it
// part of the next step's reads still hit there (measured on a 0.46 GB grid).
constexpr size_t kInfinityCacheBytes = (size_t)256 << 20;
constexpr size_t kNonTemporalBytes = 4 * kInfinityCacheBytes;
size_t step_state_bytes(const fdtd_plan* p) {
  // (the cells a step touches: row padding is never read or written)
  size_t b = (size_t)p->ncell * 49;
  for (int w = 0; w < 3; ++w) b += 6 * 4 * psi_elems(p, w);
  if (p->has_gain) b += (size_t)p->ncell * (p->gm == 2 ? 144 : 48);
  return b;
}

// z ranges of the tiles: split at the CPML slab interfaces, then into chunks.
std::vector<std::pair<int, int>> z_chunks(const fdtd_plan* p, int zchunk) {
  std::vector<int> cuts = {0};
  const int nz = p->g.nz;
  if (pml_t(p, 2) > 0) {
    // the first interior plane still reads H of the last low-side slab plane
    if (p->g.pml_lo[2] > 0 && p->g.pml_lo[2] + 1 < nz) cuts.push_back(p->g.pml_lo[2] + 1);
    if (p->g.pml_hi[2] > 0 && nz - p->g.pml_hi[2] > cuts.back()) cuts.push_back(nz - p->g.pml_hi[2]);
  }
  cuts.push_back(nz);
  // A plane in a z slab moves 81 bytes per cell instead of 49 (the two psi
  // arrays of each field), so slab segments get proportionally shorter chunks
  // and their tiles take about as long as interior tiles.
  const int zslab = std::max(1, (zchunk * 49 + 40) / 81);
  std::vector<std::pair<int, int>> out;
  for (size_t s = 0; s + 1 < cuts.size(); ++s) {
    const int a = cuts[s], b = cuts[s + 1];
    if (b <= a) continue;
    const bool in_slab = pml_t(p, 2) > 0 && ((a == 0 && p->g.pml_lo[2] > 0) || (b == nz && p->g.pml_hi[2] > 0 && a >= nz - p->g.pml_hi[2]));
    const int zc = in_slab ? zslab : zchunk;
    const int pieces = (b - a + zc - 1) / zc;
    for (int q = 0; q < pieces; ++q) {
      const int k0 = a + (int)((int64_t)(b - a) * q / pieces);
      const int k1 = a + (int)((int64_t)(b - a) * (q + 1) / pieces);
      if (k1 > k0) out.push_back({k0, k1});
    }
  }
  return out;
}

int compute_layout(fdtd_plan* p, int64_t max_steps, Layout& L) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  const size_t nc = (size_t)p->nstore;
  const int gm = gain_model_of(p->mats);
  L.desc = take(sizeof(fd_desc));
  L.mats = take(sizeof(fd_mat) * FD_MAXMAT);
  L.ninit = take(sizeof(float) * 8 * FD_MAXMAT);
  for (int b = 0; b < 2; ++b)
    for (int c = 0; c < 3; ++c) L.E[b][c] = take(nc * 4);
  for (int b = 0; b < 2; ++b)
    for (int c = 0; c < 3; ++c) L.H[b][c] = take(nc * 4);
  L.map = take(nc);
  for (int b = 0; b < 2; ++b)
    for (int c = 0; c < 3; ++c) L.P[b][c] = gm == 1 ? take(nc * 4) : 0;
  L.pop = gm ? take(nc * 4 * (gm == 2 ? 18 : 6)) : 0;
  L.gidx = gm ? take(nc * 4) : 0;
  L.glist = gm == 2 ? take(nc * 4) : 0;
  L.elist = gm == 2 ? take(nc * 4) : 0;
  for (int q = 0; q < 2; ++q) L.dmq[q] = gm == 2 ? take(nc * 4 * 3) : 0;
  for (int w = 0; w < 3; ++w) {
    const bool on = pml_t(p, w) > 0;
    L.prof[w] = on ? take(sizeof(float) * 6 * axis_n(p, w)) : 0;
    for (int f = 0; f < 2; ++f) {
      L.psiE[w][f] = on ? take(4 * psi_elems(p, w)) : 0;
      for (int b = 0; b < 2; ++b) L.psiH[b][w][f] = on ? take(4 * psi_elems(p, w)) : 0;
    }
  }
  for (size_t q = 0; q < FD_MAXSRC; ++q) {
    if (q < p->sources.size()) {
      const fdtd_source_desc& s = p->sources[q];
      const double sig = source_sigma_t(s);
      const double tend = s.delay * sig + 12.0 * sig;
      int64_t len = (int64_t)std::ceil(tend / p->dt) + 1;
      len = std::min<int64_t>(std::max<int64_t>(len, 1), std::max<int64_t>(max_steps, 1));
      p->src_len[q] = (int)len;
      L.src[q] = take(sizeof(float) * (size_t)len);
      L.srcprof[q] = s.kind == FDTD_SRC_BEAM ? take(sizeof(float) * (size_t)p->px * p->g.ny) : 0;
    } else {
      p->src_len[q] = 0;
      L.src[q] = 0;
      L.srcprof[q] = 0;
    }
  }
  const int plane = p->px * p->g.ny;  // flux-plane points, padded rows
  const int TX = p->tune.tile_x, TY = p->tune.block / p->tune.tile_x;
  p->nblk = ((p->g.nx + TX - 1) / TX) * ((p->g.ny + TY - 1) / TY);
  const auto chunks = z_chunks(p, std::max(1, p->tune.zchunk));
  p->ntiles = p->nblk * (int)chunks.size();
  L.probe = take(sizeof(float) * p->probes.size() * (size_t)std::max<int64_t>(max_steps, 1));
  for (size_t f = 0; f < FD_MAXFLUX; ++f) {
    if (f < p->flux.size()) {
      L.fluxT[f] = take(sizeof(double) * (size_t)p->nblk * (size_t)std::max<int64_t>(max_steps, 1));
      L.fluxf[f] = take(sizeof(double) * std::max<size_t>(p->flux[f].f.size(), 1));
      L.fluxacc[f] = take(sizeof(double) * 2 * 4 * p->flux[f].f.size() * (size_t)plane);
      const bool dft = !p->flux[f].f.empty();
      L.fluxring[f] = dft ? take(sizeof(float) * FD_DFT_RING * 4 * (size_t)plane) : 0;
      L.fluxprev[f] = dft ? take(sizeof(double) * 2 * 4 * p->flux[f].f.size() * (size_t)plane) : 0;
      L.fluxrot[f] = dft ? take(sizeof(double) * 6 * p->flux[f].f.size()) : 0;
    } else {
      L.fluxT[f] = L.fluxf[f] = L.fluxacc[f] = L.fluxring[f] = L.fluxprev[f] = L.fluxrot[f] = 0;
    }
  }
  L.energy = p->ke > 0 ? take(sizeof(double) * (size_t)(max_steps / p->ke + 1) * (size_t)p->ntiles) : 0;
  for (int c = 0; c < FD_NCLASS; ++c) L.tiles[c] = take(sizeof(fd_tile) * (size_t)p->ntiles);
  size_t ndft = 0;
  for (const Flux& f : p->flux)
    if (f.nf > 0) ndft += (size_t)((plane + FD_DFT_PTS - 1) / FD_DFT_PTS) * (size_t)((f.nf + FD_DFT_QB - 1) / FD_DFT_QB);
  L.dft = take(sizeof(fd_dft_tile) * std::max<size_t>(ndft, 1));
  // density-matrix pass units: cells by FD_DM_CELLS, edge range by FD_DM_EDGES,
  // one diagnostics unit per flux-plane xy tile plus one for the probes
  const size_t ndm = gm == 2 ? (nc + FD_DM_CELLS - 1) / FD_DM_CELLS + (nc + FD_DM_EDGES - 1) / FD_DM_EDGES +
                                   p->flux.size() * (size_t)p->nblk + 1
                             : 0;
  L.dmunits = take(sizeof(fd_dm_unit) * std::max<size_t>(ndm, 1));
  if (p->have_opal) {
    size_t ns = 1;
    for (int a = 0; a < 3; ++a) ns *= (size_t)(2 * p->opal.cells[a] + 1);
    L.sites = take(sizeof(int64_t) * 4 * ns);
  } else {
    L.sites = 0;
  }
  L.total = off;
  return FDTD_OK;
}

template <class T>
T* at(fdtd_plan* p, size_t off) {
  return reinterpret_cast<T*>(p->arena + off);
}

// Work units of the density-matrix passes (plans with that medium): the gain
// ordinals in runs of FD_DM_CELLS, the cells whose edges can touch a gain cell
// in runs of FD_DM_EDGES (the planes from the lowest gain plane to one past the
// highest; every plane on a periodic z axis), one diagnostics unit per xy tile
// of each flux plane and one for the probes; uploaded to the plan's arena,
// with the cells and algorithmic bytes of one launch of each pass.
int build_dm_units(fdtd_plan* p) {
  for (auto& v : p->dmu) v.clear();
  for (int q = 0; q < 4; ++q) {
    p->dm_cells[q] = 0;
    p->dm_bytes[q] = 0.0;
  }
  if (p->gm != 2) return FDTD_OK;
  const fd_desc& d = p->hdesc;
  const int ng = d.ngain;
  for (int g0 = 0; g0 < ng; g0 += FD_DM_CELLS) p->dmu[0].push_back({p->ddesc, g0, std::min(FD_DM_CELLS, ng - g0), 0});
  if (ng > 0) {
    const int plane = d.plane, nz = p->g.nz;  // padded plane of the device cell index
    const int hplane = p->g.nx * p->g.ny;     // dense plane of the host map
    int kmin = nz, kmax = -1;
    for (int k = 0; k < nz; ++k)
      for (int c = 0; c < hplane; ++c)
        if (p->mats[p->host_map[(size_t)k * hplane + c]].gain) {
          kmin = std::min(kmin, k);
          kmax = std::max(kmax, k);
          break;
        }
    const bool perz = p->g.bc[2] == FDTD_BC_PERIODIC;
    const int k0 = perz ? 0 : kmin, k1 = perz ? nz : std::min(nz, kmax + 2);
    // the edge list: cells whose own edges have a gain cell among their sharers
    // (the planes from the lowest gain plane to one past the highest), in cell
    // order, by their padded index
    std::vector<uint32_t> elist;
    const int nx = p->g.nx, ny = p->g.ny;
    auto gain_at = [&](int i, int j, int k) {
      const int n3[3] = {nx, ny, nz};
      int q[3] = {i, j, k};
      for (int a = 0; a < 3; ++a) {
        if (q[a] >= 0 && q[a] < n3[a]) continue;
        if (p->g.bc[a] != FDTD_BC_PERIODIC) return false;
        q[a] = ((q[a] % n3[a]) + n3[a]) % n3[a];
      }
      return p->mats[p->host_map[((size_t)q[2] * ny + q[1]) * nx + q[0]]].gain != 0;
    };
    for (int k = k0; k < k1; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          bool any = false;
          for (int u = 0; u < 2 && !any; ++u)
            for (int v = 0; v < 2 && !any; ++v)
              any = gain_at(i, j - u, k - v) || gain_at(i - v, j, k - u) || gain_at(i - u, j - v, k);
          if (any) elist.push_back((uint32_t)((size_t)k * plane + (size_t)j * p->px + i));
        }
    const int ne = (int)elist.size();
    if (ne)
      HIPCHK(hipMemcpy(p->arena + p->L.elist, elist.data(), sizeof(uint32_t) * elist.size(), hipMemcpyHostToDevice));
    for (int e0 = 0; e0 < ne; e0 += FD_DM_EDGES) p->dmu[1].push_back({p->ddesc, e0, std::min(FD_DM_EDGES, ne - e0), 0});
    p->dm_cells[0] = p->dm_cells[1] = ng;
    p->dm_cells[2] = ne;
    // predictor: state 72 + E^n and A of the cell's edges 24 + map and list 5
    // + Q* 12; corrector: state 72 + 72, fields 24, neighbours' Q* 12, Q 12,
    // map and list 5; edges, per listed cell: its entry 4, the sharers' Q 12,
    // A in and E out 24, its map 1
    p->dm_bytes[0] = 113.0 * ng;
    p->dm_bytes[1] = 197.0 * ng;
    p->dm_bytes[2] = 41.0 * (double)ne;
  }
  for (int f = 0; f < (int)p->flux.size(); ++f)
    for (int b = 0; b < p->nblk; ++b) p->dmu[2].push_back({p->ddesc, f, b, 0});
  p->dmu[2].push_back({p->ddesc, -1, 0, 0});
  const int64_t fpts = (int64_t)p->g.nx * p->g.ny;  // a flux plane's points (its padding is skipped)
  p->dm_cells[3] = (int64_t)p->flux.size() * fpts + (int64_t)p->probes.size();
  // E^n, E^{n+1} (x, y) and H at two planes (x, y) per flux-plane point; a probe sample
  p->dm_bytes[3] = 32.0 * (double)p->flux.size() * (double)fpts + 8.0 * (double)p->probes.size();
  p->ddm = at<fd_dm_unit>(p, p->L.dmunits);
  size_t off = 0;
  for (int q = 0; q < 3; ++q) {
    if (!p->dmu[q].empty())
      HIPCHK(hipMemcpy(p->ddm + off, p->dmu[q].data(), sizeof(fd_dm_unit) * p->dmu[q].size(), hipMemcpyHostToDevice));
    off += p->dmu[q].size();
  }
  return FDTD_OK;
}

// Enqueue one step (batch-relative index s) of the given tile sets.  With a
// Fork (graph capture) the non-empty classes become parallel graph branches.
// Density-matrix pass units of a plan or batch: cells, edges, diagnostics.
struct DmLaunch {
  const fd_dm_unit* u[3] = {nullptr, nullptr, nullptr};
  int n[3] = {0, 0, 0};
};

int enqueue_step(fd_tile* const dtiles[FD_NCLASS], const int* ntiles, const fd_xcd* part,
                 const int* pgrid, int tile_x, int block, int max_blocks, const fd_dft_tile* ddft, int ndft,
                 int maxnf, bool dft_due, int s, int ntst, const DmLaunch& dm, hipStream_t st, Fork* fk) {
  int used[FD_NCLASS], nused = 0;
  for (int c = 0; c < FD_NCLASS; ++c)
    if (ntiles[c] > 0) used[nused++] = c;
  const bool par = fk && nused > 1;
  if (par) HIPCHK(hipEventRecord(fk->fork, st));
  for (int u = 0; u < nused; ++u) {
    const int c = used[u];
    const int nt = ntiles[c];
    const int grid = max_blocks > 0 ? std::min(nt, max_blocks) : pgrid[c];
    const fd_xcd* pc = max_blocks > 0 ? nullptr : &part[c];
    hipStream_t on = st;
    if (par && u > 0) {
      on = fk->side[c];
      HIPCHK(hipStreamWaitEvent(on, fk->fork, 0));
    }
    HIPCHK(fd_launch_step(c, dtiles[c], nt, tile_x, block, grid, s, pc, ntst, on));
    if (par && u > 0) HIPCHK(hipEventRecord(fk->join[c], on));
  }
  if (par)
    for (int u = 1; u < nused; ++u) HIPCHK(hipStreamWaitEvent(st, fk->join[used[u]], 0));
  (void)maxnf;
  if (dft_due && ndft > 0) HIPCHK(fd_launch_dft(ddft, ndft, s, st));
  if (dm.n[0] > 0) HIPCHK(fd_launch_dm(dm.u[0], dm.n[0], dm.u[1], dm.n[1], dm.u[2], dm.n[2], block, s, st));
  return FDTD_OK;
}

DmLaunch plan_dm(const fdtd_plan* p) {
  DmLaunch l;
  size_t off = 0;
  for (int q = 0; q < 3; ++q) {
    l.u[q] = p->ddm ? p->ddm + off : nullptr;
    l.n[q] = (int)p->dmu[q].size();
    off += p->dmu[q].size();
  }
  return l;
}

bool plan_dft_due(const fdtd_plan* p, int64_t n) {
  for (const Flux& f : p->flux)
    if (f.nf > 0 && n % f.decim == 0) return true;
  return false;
}

int64_t plan_phase_key(const fdtd_plan* p, int64_t n0) {
  int64_t l = 1;
  for (const Flux& f : p->flux)
    if (f.nf > 0) l = std::lcm(l, (int64_t)f.decim);
  return n0 % l;
}

int plan_enqueue(fdtd_plan* p, int64_t n, hipStream_t st, Fork* fk) {
  int nt[FD_NCLASS];
  for (int c = 0; c < FD_NCLASS; ++c) nt[c] = (int)p->tiles[c].size();
  for (int64_t s = 0; s < n; ++s) {
    const int r = enqueue_step(p->dtiles, nt, p->part, p->pgrid, p->tune.tile_x, p->tune.block,
                               p->tune.max_blocks, p->ddft, (int)p->dft.size(), p->maxnf,
                               plan_dft_due(p, p->step + s), (int)s, p->ntst, plan_dm(p), st, fk);
    if (r) return r;
  }
  HIPCHK(fd_launch_advance_one(p->ddesc, n, st));
  return FDTD_OK;
}

}  // namespace

// =================================================================== ABI

extern "C" {

const char* fdtd_last_error(void) { return g_err.c_str(); }
const char* fdtd_version(void) { return "libfdtd 0.1 (gfx950)"; }

int fdtd_plan_create(const fdtd_grid_desc* g, fdtd_plan** out) {
  if (!g || !out) return fail(FDTD_EINVAL, "null argument");
  *out = nullptr;
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(FDTD_EINVAL, "grid sizes must be >= 1");
  const int64_t ncell = (int64_t)g->nx * g->ny * g->nz;
  if (ncell > (int64_t)1 << 30) return fail(FDTD_EUNSUPPORTED, "more than 2^30 cells");
  if (g->res < 1) return fail(FDTD_EINVAL, "res must be >= 1");
  if (!(g->courant > 0.0)) return fail(FDTD_EINVAL, "courant must be > 0");
  if (g->courant >= 1.0 / std::sqrt(3.0)) return fail(FDTD_EUNSTABLE, "courant %g >= 1/sqrt(3)", g->courant);
  const int n[3] = {g->nx, g->ny, g->nz};
  for (int w = 0; w < 3; ++w) {
    if (g->bc[w] != FDTD_BC_PERIODIC && g->bc[w] != FDTD_BC_PEC) return fail(FDTD_EINVAL, "bad bc on axis %d", w);
    if (g->pml_lo[w] < 0 || g->pml_hi[w] < 0) return fail(FDTD_EINVAL, "negative CPML width");
    if (g->bc[w] == FDTD_BC_PERIODIC && (g->pml_lo[w] || g->pml_hi[w]))
      return fail(FDTD_EINVAL, "CPML on a periodic axis %d", w);
    if (g->pml_lo[w] + g->pml_hi[w] > n[w]) return fail(FDTD_EINVAL, "CPML wider than the axis");
  }
  if (g->pml_lo[0] + g->pml_hi[0] + g->pml_lo[1] + g->pml_hi[1] + g->pml_lo[2] + g->pml_hi[2] > 0) {
    if (!(g->cpml_m >= 0.0) || !(g->cpml_kappa_max >= 1.0) || !(g->cpml_alpha_max >= 0.0))
      return fail(FDTD_EINVAL, "bad CPML grading parameters");
  }
  fdtd_plan* p = new (std::nothrow) fdtd_plan();
  if (!p) return fail(FDTD_ENOMEM, "host allocation");
  p->g = *g;
  p->dx = 1.0 / g->res;
  p->dt = g->courant * p->dx;
  p->ncell = ncell;
  p->px = row_pitch(g->nx);
  p->nstore = (int64_t)p->px * g->ny * g->nz;
  if (p->nstore > (int64_t)1 << 30) {
    delete p;
    return fail(FDTD_EUNSUPPORTED, "more than 2^30 cells with rows padded to %d", row_pitch(g->nx));
  }
  fdtd_material vac{};
  vac.eps = 1.0;
  p->mats.push_back(vac);
  *out = p;
  return FDTD_OK;
}

void fdtd_plan_destroy(fdtd_plan* p) {
  if (!p) return;
  for (auto& kv : p->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  if (p->cap) (void)hipStreamDestroy(p->cap);
  delete p;
}

int fdtd_set_materials(fdtd_plan* p, const fdtd_material* tab, int32_t n) {
  if (!p || !tab) return fail(FDTD_EINVAL, "null argument");
  if (p->bound) return fail(FDTD_ESTATE, "plan already bound");
  if (n < 1 || n > FDTD_MAX_MATERIALS) return fail(FDTD_EINVAL, "1..%d materials", FDTD_MAX_MATERIALS);
  for (int q = 0; q < n; ++q) {
    const fdtd_material& m = tab[q];
    if (!(m.eps > 0.0)) return fail(FDTD_EINVAL, "material %d: eps must be > 0", q);
    if (m.gain < 0 || m.gain > 2) return fail(FDTD_EINVAL, "material %d: gain must be 0, 1 or 2", q);
    if (m.gain == 1) {
      if (!(m.n_total >= 0.0) || !(m.tau32 > 0.0) || !(m.tau21 > 0.0) || !(m.tau10 > 0.0) || !(m.pump >= 0.0) ||
          !(m.f_a > 0.0) || !(m.df_a >= 0.0))
        return fail(FDTD_EINVAL, "material %d: bad gain parameters", q);
    } else if (m.gain == 2) {
      if (!(m.n_total >= 0.0) || !(m.t1 > 0.0) || !(m.t2 > 0.0) || !(m.pump >= 0.0) || !(m.f_a > 0.0))
        return fail(FDTD_EINVAL, "material %d: bad density-matrix parameters", q);
    }
    if (m.gain) {
      if (!(p->g.a_meters > 0.0)) return fail(FDTD_EINVAL, "gain needs a_meters > 0");
      for (int r = 0; r < q; ++r)
        if (tab[r].gain && tab[r].gain != m.gain)
          return fail(FDTD_EUNSUPPORTED, "materials %d and %d use different gain models", r, q);
    }
  }
  p->mats.assign(tab, tab + n);
  fd_mat scratch;
  for (int q = 0; q < n; ++q) {
    const int r = build_material(p, p->mats[q], scratch);
    if (r) return r;
  }
  return FDTD_OK;
}

int fdtd_build_opal(fdtd_plan* p, const fdtd_opal_desc* d) {
  if (!p || !d) return fail(FDTD_EINVAL, "null argument");
  if (p->bound) return fail(FDTD_ESTATE, "plan already bound");
  const int n[3] = {p->g.nx, p->g.ny, p->g.nz};
  fdg::OpalSpec o{};
  for (int a = 0; a < 3; ++a) {
    if (d->cells[a] < 1 || d->origin[a] < 0) return fail(FDTD_EINVAL, "bad opal cells/origin");
    if ((int64_t)d->origin[a] + (int64_t)d->cells[a] * p->g.res > n[a])
      return fail(FDTD_EINVAL, "opal does not fit the grid on axis %d", a);
    const bool per = p->g.bc[a] == FDTD_BC_PERIODIC;
    if (per && (d->origin[a] != 0 || d->cells[a] * p->g.res != n[a]))
      return fail(FDTD_EINVAL, "a periodic axis must be spanned by the crystal (axis %d)", a);
    o.cells[a] = d->cells[a];
    o.periodic[a] = per ? 1 : 0;
  }
  if (d->disorder < 0 || d->disorder > 2) return fail(FDTD_EINVAL, "bad disorder kind");
  if (!(d->r0 >= 0.0) || !(d->strength >= 0.0)) return fail(FDTD_EINVAL, "bad radius or strength");
  for (int m : {d->mat_bg, d->mat_void, d->mat_out})
    if (m < 0 || m >= (int)p->mats.size()) return fail(FDTD_EINVAL, "opal material index %d out of range", m);
  o.res = p->g.res;
  o.r0 = d->r0;
  o.disorder = d->disorder;
  o.strength = d->strength;
  o.seed = p->g.seed;
  o.realization = p->g.realization;
  std::vector<int64_t> rows;
  if (fdg::build_spheres(o, rows)) return fail(FDTD_EINVAL, "sphere generation failed");
  for (int a = 0; a < 3; ++a) {
    if (!o.periodic[a]) continue;
    const int64_t period = (int64_t)d->cells[a] * p->g.res * 2 * 65536;
    for (size_t s = 0; s < rows.size() / 5; ++s)
      if (2 * rows[5 * s + 4] >= period) return fail(FDTD_EINVAL, "sphere diameter reaches the period");
  }
  p->spheres.swap(rows);
  p->opal = *d;
  p->have_opal = true;
  p->map_given = false;
  return FDTD_OK;
}

int fdtd_set_material_map(fdtd_plan* p, const uint8_t* host_map) {
  if (!p || !host_map) return fail(FDTD_EINVAL, "null argument");
  if (p->bound) return fail(FDTD_ESTATE, "plan already bound");
  p->host_map.assign(host_map, host_map + p->ncell);
  p->map_given = true;
  p->have_opal = false;
  p->spheres.clear();
  return FDTD_OK;
}

int fdtd_get_spheres(const fdtd_plan* p, int64_t* out, int64_t* n) {
  if (!p || !n) return fail(FDTD_EINVAL, "null argument");
  *n = (int64_t)(p->spheres.size() / 5);
  if (out) std::memcpy(out, p->spheres.data(), p->spheres.size() * sizeof(int64_t));
  return FDTD_OK;
}

int fdtd_add_source(fdtd_plan* p, const fdtd_source_desc* s, int32_t* id) {
  if (!p || !s) return fail(FDTD_EINVAL, "null argument");
  if (p->bound) return fail(FDTD_ESTATE, "plan already bound");
  if (p->sources.size() >= FD_MAXSRC) return fail(FDTD_EINVAL, "at most %d sources", FD_MAXSRC);
  if (s->comp < 0 || s->comp > 2) return fail(FDTD_EINVAL, "source component must be 0..2");
  if (s->kind == FDTD_SRC_DIPOLE) {
    if (s->i < 0 || s->i >= p->g.nx || s->j < 0 || s->j >= p->g.ny || s->k < 0 || s->k >= p->g.nz)
      return fail(FDTD_EINVAL, "dipole outside the grid");
  } else if (s->kind == FDTD_SRC_PLANE) {
    if (s->k < 0 || s->k >= p->g.nz) return fail(FDTD_EINVAL, "source plane outside the grid");
  } else if (s->kind == FDTD_SRC_BEAM) {
    if (s->k < 0 || s->k >= p->g.nz) return fail(FDTD_EINVAL, "source plane outside the grid");
    if (!(s->waist > 0.0) || !std::isfinite(s->x0) || !std::isfinite(s->y0))
      return fail(FDTD_EINVAL, "beam waist must be > 0 and its axis finite");
  } else {
    return fail(FDTD_EINVAL, "bad source kind");
  }
  if (s->width_kind < 0 || s->width_kind > 2 || !(s->width > 0.0)) return fail(FDTD_EINVAL, "bad source width");
  p->sources.push_back(*s);
  if (id) *id = (int32_t)p->sources.size() - 1;
  return FDTD_OK;
}

int fdtd_add_probe(fdtd_plan* p, int32_t comp, int32_t i, int32_t j, int32_t k, int32_t* id) {
  if (!p) return fail(FDTD_EINVAL, "null plan");
  if (p->bound) return fail(FDTD_ESTATE, "plan already bound");
  if (p->probes.size() >= FD_MAXPROBE) return fail(FDTD_EINVAL, "at most %d probes", FD_MAXPROBE);
  if (comp < 0 || comp > 5 || i < 0 || i >= p->g.nx || j < 0 || j >= p->g.ny || k < 0 || k >= p->g.nz)
    return fail(FDTD_EINVAL, "probe outside the grid or bad component");
  p->probes.push_back({comp, i, j, k});
  if (id) *id = (int32_t)p->probes.size() - 1;
  return FDTD_OK;
}

int fdtd_add_flux_plane(fdtd_plan* p, int32_t axis, int32_t k, const double* f, int32_t nf, int32_t decim,
                        int32_t* id) {
  if (!p) return fail(FDTD_EINVAL, "null plan");
  if (p->bound) return fail(FDTD_ESTATE, "plan already bound");
  if (axis < 0 || axis > 2) return fail(FDTD_EINVAL, "flux plane axis must be 0, 1 or 2");
  if (axis != 2) return fail(FDTD_EUNSUPPORTED, "flux planes normal to z only (the output face of the crystal)");
  if (p->flux.size() >= FD_MAXFLUX) return fail(FDTD_EINVAL, "at most %d flux planes", FD_MAXFLUX);
  if (k < 0 || k >= p->g.nz || (k == 0 && p->g.bc[2] != FDTD_BC_PERIODIC))
    return fail(FDTD_EINVAL, "flux plane index out of range");
  if (nf < 0 || decim < 1 || (nf > 0 && !f)) return fail(FDTD_EINVAL, "bad frequency list or decimation");
  if (nf > 65535) return fail(FDTD_EUNSUPPORTED, "too many frequencies");
  Flux fl;
  fl.k = k;
  fl.nf = nf;
  fl.decim = decim;
  if (nf > 0) fl.f.assign(f, f + nf);
  p->flux.push_back(fl);
  if (id) *id = (int32_t)p->flux.size() - 1;
  return FDTD_OK;
}

int fdtd_set_energy_interval(fdtd_plan* p, int32_t ke) {
  if (!p) return fail(FDTD_EINVAL, "null plan");
  if (p->bound) return fail(FDTD_ESTATE, "plan already bound");
  if (ke < 0) return fail(FDTD_EINVAL, "energy interval must be >= 0");
  p->ke = ke;
  return FDTD_OK;
}

int fdtd_set_tuning(fdtd_plan* p, const fdtd_tuning* t) {
  if (!p || !t) return fail(FDTD_EINVAL, "null argument");
  if (p->bound) return fail(FDTD_ESTATE, "tuning is fixed at bind");
  if (t->block < 64 || t->block > FD_MAXBLOCK || t->block % 64) return fail(FDTD_EINVAL, "block must be 64..%d, multiple of 64", FD_MAXBLOCK);
  if (t->zchunk < 1 || t->graph_steps < 0 || t->max_blocks < 0) return fail(FDTD_EINVAL, "bad tuning");
  if (t->tile_x != 16 && t->tile_x != 32 && t->tile_x != 64) return fail(FDTD_EINVAL, "tile_x must be 16, 32 or 64");
  if (t->block % t->tile_x != 0) return fail(FDTD_EINVAL, "block must be a multiple of tile_x");
  if (2 * (t->tile_x + 2) + 2 * (t->block / t->tile_x) > t->block)
    return fail(FDTD_EINVAL, "tile_x %d with block %d: the tile's halo ring (2 (tile_x+2) + 2 block/tile_x cells) "
                "exceeds block", t->tile_x, t->block);
  if (t->merge < 0 || t->merge > 2 || t->parallel < 0 || t->parallel > 1) return fail(FDTD_EINVAL, "bad merge/parallel");
  if (t->stores < FDTD_STORES_AUTO || t->stores > FDTD_STORES_NONTEMPORAL) return fail(FDTD_EINVAL, "bad stores mode");
  if (t->cache_mb < 0) return fail(FDTD_EINVAL, "cache_mb must be >= 0");
  p->tune = *t;
  return FDTD_OK;
}

int fdtd_get_tuning(const fdtd_plan* p, fdtd_tuning* t) {
  if (!p || !t) return fail(FDTD_EINVAL, "null argument");
  *t = p->tune;
  return FDTD_OK;
}

int fdtd_required_bytes(fdtd_plan* p, int64_t max_steps, size_t* bytes) {
  if (!p || !bytes) return fail(FDTD_EINVAL, "null argument");
  if (max_steps < 0 || max_steps > ((int64_t)1 << 31)) return fail(FDTD_EINVAL, "max_steps out of range");
  Layout L;
  const int r = compute_layout(p, max_steps, L);
  if (r) return r;
  *bytes = L.total;
  return FDTD_OK;
}

int fdtd_bind_arena(fdtd_plan* p, void* dev, size_t bytes, int64_t max_steps, void* stream) {
  if (!p || !dev) return fail(FDTD_EINVAL, "null argument");
  if (p->bound) return fail(FDTD_ESTATE, "plan already bound");
  if (((uintptr_t)dev & 255) != 0) return fail(FDTD_EINVAL, "arena must be 256-byte aligned");
  if (max_steps < 0 || max_steps > ((int64_t)1 << 31)) return fail(FDTD_EINVAL, "max_steps out of range");
  hipStream_t st = (hipStream_t)stream;
  Layout L;
  int r = compute_layout(p, max_steps, L);
  if (r) return r;
  if (bytes < L.total) return fail(FDTD_ENOMEM, "arena of %zu bytes, need %zu", bytes, L.total);
  if (!p->have_opal && !p->map_given) p->host_map.assign((size_t)p->ncell, 0);
  if (p->map_given || !p->have_opal)
    for (uint8_t m : p->host_map)
      if (m >= p->mats.size()) return fail(FDTD_EINVAL, "material map index %d out of range", (int)m);
  p->arena = (uint8_t*)dev;
  p->arena_bytes = bytes;
  p->max_steps = max_steps;
  p->L = L;
  HIPCHK(fd_launch_fill(dev, L.total, st));

  // materials
  std::vector<fd_mat> mt(FD_MAXMAT);
  // initial populations per material as FP32 (hi, lo) pairs: hi + lo is n_init
  // to about 48 bits, as the state stores them
  std::vector<float> ninit(8 * FD_MAXMAT, 0.0f);
  p->has_gain = false;
  p->gm = gain_model_of(p->mats);
  for (size_t q = 0; q < p->mats.size(); ++q) {
    r = build_material(p, p->mats[q], mt[q]);
    if (r) return r;
    if (p->mats[q].gain) {
      p->has_gain = true;
      for (int l = 0; l < 4; ++l) {
        const float hi = (float)p->mats[q].n_init[l];
        ninit[8 * q + l] = hi;
        ninit[8 * q + 4 + l] = (float)(p->mats[q].n_init[l] - (double)hi);
      }
    }
  }
  HIPCHK(hipMemcpyAsync(p->arena + L.mats, mt.data(), sizeof(fd_mat) * FD_MAXMAT, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->arena + L.ninit, ninit.data(), sizeof(float) * ninit.size(), hipMemcpyHostToDevice, st));

  // descriptor
  fd_desc& d = p->hdesc;
  std::memset(&d, 0, sizeof d);
  d.nx = p->g.nx; d.ny = p->g.ny; d.nz = p->g.nz;
  d.px = p->px;
  d.plane = p->px * p->g.ny;
  for (int w = 0; w < 3; ++w) d.per[w] = p->g.bc[w] == FDTD_BC_PERIODIC ? 1 : 0;
  d.ncell = (int)p->nstore;
  d.ch = (float)(p->dt / p->dx);
  d.nmat = (int)p->mats.size();
  d.has_gain = p->has_gain ? 1 : 0;
  d.gain_model = p->gm;
  d.gainmask = 0u;
  for (size_t m = 0; m < p->mats.size(); ++m)
    if (p->mats[m].gain) d.gainmask |= 1u << m;
  d.block = p->tune.block;
  d.step = 0;
  d.max_steps = max_steps;
  d.mats = at<fd_mat>(p, L.mats);
  d.mat = at<uint8_t>(p, L.map);
  for (int b = 0; b < 2; ++b)
    for (int c = 0; c < 3; ++c) {
      d.E[b][c] = at<float>(p, L.E[b][c]);
      d.H[b][c] = at<float>(p, L.H[b][c]);
      d.P[b][c] = p->gm == 1 ? at<float>(p, L.P[b][c]) : nullptr;
    }
  d.pop = p->has_gain ? at<float>(p, L.pop) : nullptr;
  d.gidx = p->has_gain ? at<uint32_t>(p, L.gidx) : nullptr;
  d.glist = p->gm == 2 ? at<uint32_t>(p, L.glist) : nullptr;
  d.elist = p->gm == 2 ? at<uint32_t>(p, L.elist) : nullptr;
  for (int q = 0; q < 2; ++q) d.dmq[q] = p->gm == 2 ? at<float>(p, L.dmq[q]) : nullptr;
  d.tile_x = p->tune.tile_x;
  d.key0 = p->g.seed;
  d.key1 = p->g.realization;
  std::vector<float> prof;
  for (int w = 0; w < 3; ++w) {
    d.pml_t[w] = pml_t(p, w);
    d.pml_lo[w] = d.pml_t[w] ? p->g.pml_lo[w] : 0;
    d.pml_hi[w] = d.pml_t[w] ? p->g.pml_hi[w] : 0;
    if (!d.pml_t[w]) continue;
    const int nw = axis_n(p, w);
    prof.assign((size_t)6 * nw, 0.0f);
    for (int q = 0; q < nw; ++q) {
      cpml_point(p, w, (double)q, prof[q], prof[nw + q], prof[2 * nw + q]);
      cpml_point(p, w, (double)q + 0.5, prof[3 * nw + q], prof[4 * nw + q], prof[5 * nw + q]);
    }
    HIPCHK(hipMemcpyAsync(p->arena + L.prof[w], prof.data(), sizeof(float) * prof.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    d.prof[w] = at<float>(p, L.prof[w]);
    for (int f = 0; f < 2; ++f) {
      d.psiE[w][f] = at<float>(p, L.psiE[w][f]);
      for (int b = 0; b < 2; ++b) d.psiH[b][w][f] = at<float>(p, L.psiH[b][w][f]);
    }
  }
  // sources
  d.nsrc = (int)p->sources.size();
  for (int q = 0; q < d.nsrc; ++q) {
    const fdtd_source_desc& s = p->sources[q];
    const double sig = source_sigma_t(s);
    const double t0 = s.delay * sig;
    std::vector<float> tab((size_t)p->src_len[q]);
    for (int64_t n = 0; n < p->src_len[q]; ++n) {
      const double t = ((double)n + 0.5) * p->dt - t0;
      const double v = s.amp * std::sin(2.0 * kPi * s.f0 * t) * std::exp(-t * t / (2.0 * sig * sig));
      tab[(size_t)n] = (float)(s.kind == FDTD_SRC_DIPOLE ? v / (p->dx * p->dx) : v);
    }
    HIPCHK(hipMemcpyAsync(p->arena + L.src[q], tab.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    d.src_kind[q] = s.kind;
    d.src_comp[q] = s.comp;
    d.src_k[q] = s.k;
    d.src_cell[q] = s.kind == FDTD_SRC_DIPOLE ? s.j * p->px + s.i : -1;
    d.src_len[q] = p->src_len[q];
    d.src_tab[q] = at<float>(p, L.src[q]);
    d.src_prof[q] = nullptr;
    if (s.kind == FDTD_SRC_BEAM) {
      // TEM00 waist profile at the driven component's Yee position (FP64, stored FP32)
      std::vector<float> prof((size_t)p->px * p->g.ny, 0.0f);
      for (int j = 0; j < p->g.ny; ++j)
        for (int i = 0; i < p->g.nx; ++i) {
          const double x = ((double)i + (s.comp == 0 ? 0.5 : 0.0)) * p->dx;
          const double y = ((double)j + (s.comp == 1 ? 0.5 : 0.0)) * p->dx;
          const double rx = x - s.x0, ry = y - s.y0;
          prof[(size_t)j * p->px + i] = (float)std::exp(-(rx * rx + ry * ry) / (s.waist * s.waist));
        }
      HIPCHK(hipMemcpyAsync(p->arena + L.srcprof[q], prof.data(), sizeof(float) * prof.size(),
                            hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
      d.src_prof[q] = at<float>(p, L.srcprof[q]);
    }
  }
  // probes
  d.nprobe = (int)p->probes.size();
  for (int q = 0; q < d.nprobe; ++q) {
    d.probe_comp[q] = p->probes[q][0];
    d.probe_cell[q] = p->probes[q][2] * p->px + p->probes[q][1];
    d.probe_k[q] = p->probes[q][3];
  }
  d.probe_ring = at<float>(p, L.probe);
  // flux
  d.nflux = (int)p->flux.size();
  d.nblk = p->nblk;
  p->maxnf = 0;
  for (int f = 0; f < d.nflux; ++f) {
    const Flux& fl = p->flux[f];
    d.flux_k[f] = fl.k;
    d.flux_T[f] = at<double>(p, L.fluxT[f]);
    d.flux_nf[f] = fl.nf;
    d.flux_decim[f] = fl.decim;
    d.flux_f[f] = at<double>(p, L.fluxf[f]);
    d.flux_acc[f] = at<double>(p, L.fluxacc[f]);
    d.flux_ring[f] = fl.nf > 0 ? at<float>(p, L.fluxring[f]) : nullptr;
    d.flux_prev[f] = fl.nf > 0 ? at<double>(p, L.fluxprev[f]) : nullptr;
    d.flux_rot[f] = fl.nf > 0 ? at<double>(p, L.fluxrot[f]) : nullptr;
    if (fl.nf > 0) {
      // unit phasors of one ring, one sample interval and half a step, per frequency
      std::vector<double> rot(6 * (size_t)fl.nf);
      for (int q = 0; q < fl.nf; ++q) {
        const double w = 2.0 * kPi * fl.f[(size_t)q] * p->dt;
        const double a[3] = {w * (double)fl.decim * FD_DFT_RING, w * (double)fl.decim, 0.5 * w};
        for (int r = 0; r < 3; ++r) {
          rot[6 * (size_t)q + 2 * r] = std::cos(a[r]);
          rot[6 * (size_t)q + 2 * r + 1] = std::sin(a[r]);
        }
      }
      HIPCHK(hipMemcpyAsync(p->arena + L.fluxrot[f], rot.data(), sizeof(double) * rot.size(), hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    if (fl.nf > 0) {
      HIPCHK(hipMemcpyAsync(p->arena + L.fluxf[f], fl.f.data(), sizeof(double) * fl.nf, hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    p->maxnf = std::max(p->maxnf, fl.nf);
  }
  d.ke = p->ke;
  d.ntiles = p->ntiles;
  d.energy = p->ke > 0 ? at<double>(p, L.energy) : nullptr;
  d.dt = p->dt;
  p->ddesc = at<fd_desc>(p, L.desc);
  HIPCHK(hipMemcpyAsync(p->ddesc, &d, sizeof d, hipMemcpyHostToDevice, st));

  // material map: given, or voxelized from the sphere list on the device
  if (p->have_opal) {
    const fdtd_opal_desc& o = p->opal;
    int ext[3], per[3], ncr[3];
    for (int a = 0; a < 3; ++a) {
      per[a] = p->g.bc[a] == FDTD_BC_PERIODIC ? 1 : 0;
      ext[a] = 2 * o.cells[a] + (per[a] ? 0 : 1);
      ncr[a] = o.cells[a] * p->g.res;
    }
    const size_t nsite = (size_t)ext[0] * ext[1] * ext[2];
    std::vector<int64_t> sites(4 * nsite, 0);
    for (size_t q = 0; q < nsite; ++q) sites[4 * q + 3] = -1;
    int64_t reach[3] = {0, 0, 0};
    const int64_t half_site = (int64_t)p->g.res * 65536;  // quanta between half-lattice sites
    const int64_t wx = 2 * (int64_t)o.cells[0] + 1, wy = 2 * (int64_t)o.cells[1] + 1;
    for (size_t s = 0; s < p->spheres.size() / 5; ++s) {
      const int64_t* row = &p->spheres[5 * s];
      const int64_t id = row[0];
      const int64_t h = id % wx, kk = (id / wx) % wy, l = id / (wx * wy);
      const int64_t hv[3] = {h, kk, l};
      const size_t q = (size_t)((l * ext[1] + kk) * ext[0] + h);
      for (int a = 0; a < 3; ++a) sites[4 * q + a] = row[1 + a];
      sites[4 * q + 3] = row[4];
      for (int a = 0; a < 3; ++a) {
        const int64_t dev_a = std::llabs(row[1 + a] - hv[a] * half_site);
        reach[a] = std::max(reach[a], row[4] + dev_a);
      }
    }
    HIPCHK(hipMemcpyAsync(p->arena + L.sites, sites.data(), sizeof(int64_t) * sites.size(), hipMemcpyHostToDevice, st));
    HIPCHK(fd_launch_voxelize(at<int64_t>(p, L.sites), ext[0], ext[1], ext[2], per, ncr, o.origin, reach, p->g.res,
                              o.mat_bg, o.mat_void, o.mat_out, p->g.nx, p->g.ny, p->g.nz, p->px,
                              at<uint8_t>(p, L.map), st));
    p->host_map.resize((size_t)p->ncell);
    HIPCHK(copy_rows_to_host(p, p->host_map.data(), p->arena + L.map, 1, st));
    HIPCHK(hipStreamSynchronize(st));
  } else {
    HIPCHK(copy_rows_to_device(p, p->arena + L.map, p->host_map.data(), 1, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  if (p->has_gain) {
    // gain ordinals (gain cells numbered in cell order) and the initial
    // populations at them; the rest of the state starts at zero with the arena
    // (the order of cells is the same in the dense and the padded layout)
    const size_t nc = (size_t)p->ncell;
    p->gidx.assign(nc, 0u);
    uint32_t g = 0;
    for (size_t o = 0; o < nc; ++o)
      if (p->mats[p->host_map[o]].gain) p->gidx[o] = g++;
    HIPCHK(copy_rows_to_device(p, p->arena + L.gidx, p->gidx.data(), sizeof(uint32_t), st));
    HIPCHK(fd_launch_init_pop(at<uint8_t>(p, L.map), at<float>(p, L.ninit), at<uint32_t>(p, L.gidx), d.gainmask,
                              d.pop, d.ncell, d.nx, d.px, st));
    HIPCHK(hipStreamSynchronize(st));
    d.ngain = (int)g;
    if (p->gm == 2) {
      // the (padded) cell of each gain ordinal, for the density-matrix passes
      std::vector<uint32_t> glist(g);
      for (size_t o = 0; o < nc; ++o)
        if (p->mats[p->host_map[o]].gain) glist[p->gidx[o]] = (uint32_t)pitched(p, o);
      if (g) HIPCHK(hipMemcpyAsync(p->arena + L.glist, glist.data(), sizeof(uint32_t) * g, hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipMemcpyAsync(p->ddesc, &d, sizeof d, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }

  // tiles, classified by CPML and gain presence
  const int plane = p->g.nx * p->g.ny;  // dense plane of the host map
  const int TX = p->tune.tile_x, TY = p->tune.block / p->tune.tile_x;
  const int ntx = (p->g.nx + TX - 1) / TX, nty = (p->g.ny + TY - 1) / TY;
  const auto chunks = z_chunks(p, std::max(1, p->tune.zchunk));
  std::vector<uint8_t> gain_mat(FD_MAXMAT, 0);
  for (size_t q = 0; q < p->mats.size(); ++q) gain_mat[q] = p->mats[q].gain ? 1 : 0;
  // gain cells per (xy tile, z)
  std::vector<int> blk_gain;
  if (p->has_gain) {
    blk_gain.assign((size_t)p->nblk * p->g.nz, 0);
    for (int k = 0; k < p->g.nz; ++k)
      for (int j = 0; j < p->g.ny; ++j)
        for (int i = 0; i < p->g.nx; ++i)
          if (gain_mat[p->host_map[(size_t)k * plane + (size_t)j * p->g.nx + i]])
            blk_gain[(size_t)k * p->nblk + (size_t)(j / TY) * ntx + i / TX] += 1;
  }
  // cells of [a, b) inside the slabs of axis w
  auto slab_count = [&](int w, int a, int b) {
    if (!d.pml_t[w]) return 0;
    const int n = w == 0 ? p->g.nx : (w == 1 ? p->g.ny : p->g.nz);
    const int lo = std::max(0, std::min(b, d.pml_lo[w]) - a);
    const int hi = std::max(0, b - std::max(a, n - d.pml_hi[w]));
    return lo + hi;
  };
  for (int c = 0; c < FD_NCLASS; ++c) {
    p->tiles[c].clear();
    p->tcost[c].clear();
  }
  std::vector<fd_tile> all;
  std::vector<double> tcost;
  std::vector<std::pair<int, int>> tcls;
  int tidx = 0;
  for (const auto& ch : chunks) {
    for (int by = 0; by < nty; ++by)
      for (int bx = 0; bx < ntx; ++bx) {
        fd_tile t{};
        t.d = p->ddesc;
        t.i0 = bx * TX;
        t.j0 = by * TY;
        t.k0 = ch.first;
        t.k1 = ch.second;
        t.tidx = tidx++;
        t.blk = by * ntx + bx;
        // sources, probes and flux planes the tile's kernel must look at
        for (int q = 0; q < d.nsrc; ++q) {
          if (d.src_k[q] < t.k0 || d.src_k[q] >= t.k1) continue;
          if (d.src_kind[q] == FDTD_SRC_DIPOLE) {
            const int si = d.src_cell[q] % p->px, sj = d.src_cell[q] / p->px;
            if (si < t.i0 || si >= t.i0 + TX || sj < t.j0 || sj >= t.j0 + TY) continue;
          }
          t.srcmask |= 1u << q;
        }
        for (int q = 0; q < d.nprobe; ++q) {
          const int pi = d.probe_cell[q] % p->px, pj = d.probe_cell[q] / p->px;
          if (d.probe_k[q] >= t.k0 && d.probe_k[q] < t.k1 && pi >= t.i0 && pi < t.i0 + TX && pj >= t.j0 &&
              pj < t.j0 + TY)
            t.pmask |= 1u << q;
        }
        for (int q = 0; q < d.nflux; ++q)
          if (d.flux_k[q] >= t.k0 && d.flux_k[q] < t.k1) t.fmask |= 1u << q;
        if (d.pml_t[2] && (t.k0 < d.pml_lo[2] || t.k1 > p->g.nz - d.pml_hi[2])) t.flags |= FD_TILE_ZSLAB;
        // A tile needs the CPML code if any H value it evaluates lies in a slab:
        // its own cells, the x-1 / y-1 neighbours it recomputes, and plane k0-1.
        // (Slabs only exist on PEC axes, so no wrap-around is involved.)
        int axes = 0;
        if (d.pml_t[2] && (t.k0 - 1 < d.pml_lo[2] || t.k1 > p->g.nz - d.pml_hi[2])) axes |= 4;
        const int iend = std::min(p->g.nx, t.i0 + TX), jend = std::min(p->g.ny, t.j0 + TY);
        if (d.pml_t[0] && (t.i0 - 1 < d.pml_lo[0] || iend > p->g.nx - d.pml_hi[0])) axes |= 1;
        if (d.pml_t[1] && (t.j0 - 1 < d.pml_lo[1] || jend > p->g.ny - d.pml_hi[1])) axes |= 2;
        int pml = axes == 0 ? 0 : (axes == 4 ? 1 : 2);
        long long ngain = 0;
        if (p->has_gain)
          for (int k = t.k0; k < t.k1; ++k) ngain += blk_gain[(size_t)k * p->nblk + t.blk];
        // density-matrix plans step with the classes without gain: the matter
        // has passes of its own after the step kernels
        const bool gain = ngain > 0 && p->gm != 2;
        const int nxt_ = iend - t.i0, nyt_ = jend - t.j0, nzt_ = t.k1 - t.k0;
        const double slab_cells = (double)slab_count(0, t.i0, iend) * nyt_ * nzt_ +
                                  (double)nxt_ * slab_count(1, t.j0, jend) * nzt_ +
                                  (double)nxt_ * nyt_ * slab_count(2, t.k0, t.k1);
        // algorithmic bytes of the tile, plus the plane below it that it also stages
        tcost.push_back(49.0 * nxt_ * nyt_ * (nzt_ + 1) + 32.0 * slab_cells + (gain ? 84.0 * (double)ngain : 0.0));
        tcls.push_back({pml, gain ? 1 : 0});
        all.push_back(t);
      }
  }
  // fold classes into fewer launches: a more general kernel is correct on a
  // simpler tile (slab and gain tests are per cell / per plane at run time)
  int max_pml = 0, any_gain = 0;
  for (const auto& pc : tcls) {
    max_pml = std::max(max_pml, pc.first);
    any_gain |= pc.second;
  }
  for (size_t q = 0; q < all.size(); ++q) {
    int pml = tcls[q].first, gain = tcls[q].second;
    if (p->tune.merge >= 1 && pml == 0 && d.pml_t[2]) pml = 1;
    if (p->tune.merge >= 2) {
      pml = max_pml;
      gain = any_gain;
    }
    p->tiles[pml + 3 * gain].push_back(all[q]);
    p->tcost[pml + 3 * gain].push_back(tcost[q]);
  }
  for (int c = 0; c < FD_NCLASS; ++c) p->part[c] = xcd_partition(p->tcost[c], &p->pgrid[c]);
  for (int c = 0; c < FD_NCLASS; ++c) {
    p->dtiles[c] = at<fd_tile>(p, L.tiles[c]);
    if (!p->tiles[c].empty())
      HIPCHK(hipMemcpyAsync(p->dtiles[c], p->tiles[c].data(), sizeof(fd_tile) * p->tiles[c].size(),
                            hipMemcpyHostToDevice, st));
  }
  p->dft.clear();
  for (int f = 0; f < d.nflux; ++f) {
    if (p->flux[f].nf == 0) continue;
    for (int p0 = 0; p0 < d.plane; p0 += FD_DFT_PTS)  // the padded plane's points
      for (int q0 = 0; q0 < p->flux[f].nf; q0 += FD_DFT_QB) {
        fd_dft_tile t{};
        t.d = p->ddesc;
        t.flux = f;
        t.p0 = p0;
        t.q0 = q0;
        p->dft.push_back(t);
      }
  }
  p->ddft = at<fd_dft_tile>(p, L.dft);
  if (!p->dft.empty())
    HIPCHK(hipMemcpyAsync(p->ddft, p->dft.data(), sizeof(fd_dft_tile) * p->dft.size(), hipMemcpyHostToDevice, st));
  if (int r = build_dm_units(p)) return r;
  HIPCHK(hipStreamSynchronize(st));
  p->step = 0;
  p->ntst = p->tune.stores == FDTD_STORES_NONTEMPORAL ? 1
            : p->tune.stores == FDTD_STORES_ORDINARY ? 0
            : (step_state_bytes(p) > kNonTemporalBytes ? 1 : 0);
  p->bound = true;
  return FDTD_OK;
}

int fdtd_get_material_map(fdtd_plan* p, uint8_t* host_map, void* stream) {
  if (!p || !host_map) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(copy_rows_to_host(p, host_map, p->arena + p->L.map, 1, st));
  HIPCHK(hipStreamSynchronize(st));
  return FDTD_OK;
}

static int plan_step(fdtd_plan* p, int64_t n, hipStream_t st) {
  if (n < 0) return fail(FDTD_EINVAL, "negative step count");
  if (p->step + n > p->max_steps) return fail(FDTD_ESTATE, "max_steps (%lld) exceeded", (long long)p->max_steps);
  const int64_t K = p->tune.graph_steps;
  int64_t done = 0;
  if (K > 0) {
    while (n - done >= K) {
      const int64_t key = plan_phase_key(p, p->step) * 1000003 + K;
      auto it = p->graphs.find(key);
      if (it == p->graphs.end()) {
        if (!p->cap) HIPCHK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
        Fork* fk = nullptr;
        if (p->tune.parallel) {
          if (!p->fork) p->fork.reset(new Fork());
          if (int rf = p->fork->init()) return rf;
          fk = p->fork.get();
        }
        GraphEntry ge;
        HIPCHK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
        const int r = plan_enqueue(p, K, p->cap, fk);
        hipGraph_t gr = nullptr;
        const hipError_t e = hipStreamEndCapture(p->cap, &gr);
        if (r) {
          if (gr) (void)hipGraphDestroy(gr);
          return r;
        }
        if (e != hipSuccess) return fail(FDTD_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        ge.graph = gr;
        HIPCHK(hipGraphInstantiate(&ge.exec, gr, nullptr, nullptr, 0));
        it = p->graphs.emplace(key, ge).first;
      }
      HIPCHK(hipGraphLaunch(it->second.exec, st));
      p->step += K;
      done += K;
    }
  }
  if (n - done > 0) {
    const int r = plan_enqueue(p, n - done, st, nullptr);
    if (r) return r;
    p->step += n - done;
  }
  return FDTD_OK;
}

int fdtd_step(fdtd_plan* p, int64_t n, void* stream) {
  if (!p) return fail(FDTD_EINVAL, "null plan");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  return plan_step(p, n, (hipStream_t)stream);
}

int64_t fdtd_step_count(const fdtd_plan* p) { return p ? p->step : -1; }
int64_t fdtd_cell_count(const fdtd_plan* p) { return p ? p->ncell : -1; }
double fdtd_dt(const fdtd_plan* p) { return p ? p->dt : 0.0; }

int fdtd_read_field(fdtd_plan* p, int32_t comp, float* host, void* stream) {
  if (!p || !host) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  if (comp < 0 || comp > 5) return fail(FDTD_EINVAL, "component must be 0..5");
  hipStream_t st = (hipStream_t)stream;
  const int par = (int)(p->step & 1);
  const size_t off = comp < 3 ? p->L.E[par][comp] : p->L.H[par][comp - 3];
  HIPCHK(copy_rows_to_host(p, host, p->arena + off, sizeof(float), st));
  HIPCHK(hipStreamSynchronize(st));
  return FDTD_OK;
}

int fdtd_write_field(fdtd_plan* p, int32_t comp, const float* host, void* stream) {
  if (!p || !host) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  if (comp < 0 || comp > 5) return fail(FDTD_EINVAL, "component must be 0..5");
  hipStream_t st = (hipStream_t)stream;
  const int par = (int)(p->step & 1);
  const size_t off = comp < 3 ? p->L.E[par][comp] : p->L.H[par][comp - 3];
  HIPCHK(copy_rows_to_device(p, p->arena + off, host, sizeof(float), st));
  HIPCHK(hipStreamSynchronize(st));
  return FDTD_OK;
}

int fdtd_read_probe(fdtd_plan* p, int32_t id, float* host, int64_t* n, void* stream) {
  if (!p || !host) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  if (id < 0 || id >= (int)p->probes.size()) return fail(FDTD_EINVAL, "bad probe id");
  hipStream_t st = (hipStream_t)stream;
  if (p->step > 0)
    HIPCHK(hipMemcpyAsync(host, p->arena + p->L.probe + sizeof(float) * (size_t)id * (size_t)p->max_steps,
                          sizeof(float) * (size_t)p->step, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (n) *n = p->step;
  return FDTD_OK;
}

int fdtd_read_flux(fdtd_plan* p, int32_t id, double* T, double* spec, int64_t* n, void* stream) {
  if (!p) return fail(FDTD_EINVAL, "null plan");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  if (id < 0 || id >= (int)p->flux.size()) return fail(FDTD_EINVAL, "bad flux id");
  hipStream_t st = (hipStream_t)stream;
  const double dx2 = p->dx * p->dx;
  if (T && p->step > 0) {
    std::vector<double> part((size_t)p->step * p->nblk);
    HIPCHK(hipMemcpyAsync(part.data(), p->arena + p->L.fluxT[id], sizeof(double) * part.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int64_t s = 0; s < p->step; ++s) {
      double acc = 0.0;
      for (int b = 0; b < p->nblk; ++b) acc += part[(size_t)s * p->nblk + b];
      T[s] = acc * dx2;
    }
  }
  const Flux& fl = p->flux[id];
  if (spec && fl.nf > 0) {
    const size_t plane = (size_t)p->px * p->g.ny;  // padded points (their sums stay 0)
    std::vector<double> acc(2 * 4 * (size_t)fl.nf * plane);
    // samples taken at steps 0, decim, ... < step; complete rings are already in
    // the sums, the rest is added into a copy
    const int64_t nsamp = (p->step + fl.decim - 1) / fl.decim;
    const int pending = (int)(nsamp % FD_DFT_RING);
    size_t src = p->L.fluxacc[id];
    if (pending > 0) {
      HIPCHK(fd_launch_dft_preview(p->ddft, (int)p->dft.size(), id, nsamp - pending, pending, st));
      src = p->L.fluxprev[id];
    }
    HIPCHK(hipMemcpyAsync(acc.data(), p->arena + src, sizeof(double) * acc.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int q = 0; q < fl.nf; ++q) {
      double sum = 0.0;
      for (size_t pt = 0; pt < plane; ++pt) {
        const double* ex = &acc[2 * ((0 * (size_t)fl.nf + q) * plane + pt)];
        const double* ey = &acc[2 * ((1 * (size_t)fl.nf + q) * plane + pt)];
        const double* hx = &acc[2 * ((2 * (size_t)fl.nf + q) * plane + pt)];
        const double* hy = &acc[2 * ((3 * (size_t)fl.nf + q) * plane + pt)];
        sum += (ex[0] * hy[0] + ex[1] * hy[1]) - (ey[0] * hx[0] + ey[1] * hx[1]);
      }
      spec[q] = sum * dx2;
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  if (n) *n = p->step;
  return FDTD_OK;
}

int fdtd_read_populations(fdtd_plan* p, double* host, void* stream) {
  if (!p || !host) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  if (!p->has_gain) return fail(FDTD_ESTATE, "no gain material");
  hipStream_t st = (hipStream_t)stream;
  const size_t nc = (size_t)p->ncell, ns = (size_t)p->nstore;  // host and device plane strides
  std::vector<float> pop(6 * ns);
  HIPCHK(hipMemcpyAsync(pop.data(), p->arena + p->L.pop, sizeof(float) * pop.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (size_t o = 0; o < nc; ++o) {
    if (!p->mats[p->host_map[o]].gain) {
      for (int l = 0; l < 4; ++l) host[l * nc + o] = 0.0;
      continue;
    }
    const size_t q = p->gidx[o];  // state index of the cell
    double lv[3];  // hi + lo of each pair: exact in FP64
    for (int l = 0; l < 3; ++l) lv[l] = (double)pop[l * ns + q] + (double)pop[(3 + l) * ns + q];
    host[0 * nc + o] = 1.0 - (lv[0] + lv[1] + lv[2]);
    for (int l = 0; l < 3; ++l) host[(1 + l) * nc + o] = lv[l];
  }
  return FDTD_OK;
}

int fdtd_read_polarization(fdtd_plan* p, float* host, void* stream) {
  if (!p || !host) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  if (!p->has_gain) return fail(FDTD_ESTATE, "no gain material");
  hipStream_t st = (hipStream_t)stream;
  const size_t nc = (size_t)p->ncell, ns = (size_t)p->nstore;
  if (p->gm == 2) {  // P_c = 2 kappa Re rho_0c of each gain cell's material
    std::vector<float> re(3 * ns);
    HIPCHK(hipMemcpyAsync(re.data(), p->arena + p->L.pop + sizeof(float) * 6 * ns, sizeof(float) * re.size(),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<float> k2(p->mats.size(), 0.0f);
    for (size_t m = 0; m < p->mats.size(); ++m) {
      fd_mat mt;
      if (p->mats[m].gain && build_material(p, p->mats[m], mt) == FDTD_OK) k2[m] = mt.bk2;
    }
    for (int c = 0; c < 3; ++c)
      for (size_t o = 0; o < nc; ++o) host[c * nc + o] = k2[p->host_map[o]] * re[c * ns + p->gidx[o]];
    return FDTD_OK;
  }
  const int par = (int)(p->step & 1);
  std::vector<float> pb(3 * nc);
  for (int c = 0; c < 3; ++c)
    HIPCHK(hipMemcpyAsync(pb.data() + (size_t)c * nc, p->arena + p->L.P[par][c], sizeof(float) * nc,
                          hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int c = 0; c < 3; ++c)
    for (size_t o = 0; o < nc; ++o) host[c * nc + o] = p->mats[p->host_map[o]].gain ? pb[c * nc + p->gidx[o]] : 0.0f;
  return FDTD_OK;
}

int fdtd_read_density(fdtd_plan* p, float* host, void* stream) {
  if (!p || !host) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  if (p->gm != 2) return fail(FDTD_ESTATE, "no density-matrix gain material");
  hipStream_t st = (hipStream_t)stream;
  const size_t nc = (size_t)p->ncell;
  const size_t ns = (size_t)p->nstore;
  std::vector<float> st18(18 * ns);
  HIPCHK(hipMemcpyAsync(st18.data(), p->arena + p->L.pop, sizeof(float) * st18.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (size_t o = 0; o < nc; ++o) {
    const bool g = p->mats[p->host_map[o]].gain != 0;
    const size_t q = p->gidx[o];
    for (int l = 0; l < 3; ++l)
      host[l * nc + o] = g ? (float)((double)st18[l * ns + q] + (double)st18[(3 + l) * ns + q]) : 0.0f;
    for (int l = 3; l < 15; ++l) host[l * nc + o] = g ? st18[(3 + l) * ns + q] : 0.0f;
  }
  return FDTD_OK;
}

int fdtd_read_energy(fdtd_plan* p, double* host, int64_t* n, void* stream) {
  if (!p || !host || !n) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  if (p->ke <= 0) return fail(FDTD_ESTATE, "energy not enabled");
  hipStream_t st = (hipStream_t)stream;
  const int64_t ns = (p->step + p->ke - 1) / p->ke;
  if (ns > 0) {
    std::vector<double> part((size_t)ns * p->ntiles);
    HIPCHK(hipMemcpyAsync(part.data(), p->arena + p->L.energy, sizeof(double) * part.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double w = 0.5 * p->dx * p->dx * p->dx;
    for (int64_t s = 0; s < ns; ++s) {
      double acc = 0.0;
      for (int t = 0; t < p->ntiles; ++t) acc += part[(size_t)s * p->ntiles + t];
      host[s] = acc * w;
    }
  }
  *n = ns;
  return FDTD_OK;
}

int fdtd_time_steps(fdtd_plan* p, int64_t n, void* stream, double* ms) {
  if (!p || !ms) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  HIPCHK(hipEventRecord(a, st));
  int r = plan_step(p, n, st);
  if (r) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return r;
  }
  HIPCHK(hipEventRecord(b, st));
  HIPCHK(hipEventSynchronize(b));
  float f = 0.0f;
  HIPCHK(hipEventElapsedTime(&f, a, b));
  *ms = f;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return FDTD_OK;
}

int fdtd_class_cells(const fdtd_plan* p, int64_t* cells) {
  if (!p || !cells) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  const int plane = p->g.nx * p->g.ny;
  const int TX = p->tune.tile_x, TY = p->tune.block / p->tune.tile_x;
  for (int c = 0; c < FD_NCLASS; ++c) {
    int64_t acc = 0;
    for (const fd_tile& t : p->tiles[c])
      acc += (int64_t)std::min(TX, p->g.nx - t.i0) * std::min(TY, p->g.ny - t.j0) * (t.k1 - t.k0);
    cells[c] = acc;
  }
  int64_t pts = 0;
  for (const Flux& f : p->flux)
    if (f.nf > 0) pts += plane;
  cells[FD_KERNEL_DFT] = pts;
  for (int q = 0; q < 4; ++q) cells[FD_KERNEL_DM + q] = p->dm_cells[q];
  return FDTD_OK;
}

int fdtd_class_bytes(const fdtd_plan* p, double* bytes) {
  if (!p || !bytes) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  const int nx = p->g.nx, ny = p->g.ny, nz = p->g.nz;
  const int TX = p->tune.tile_x, TY = p->tune.block / p->tune.tile_x;
  auto in_slab = [&](int w, int q) {
    const int n = w == 0 ? nx : (w == 1 ? ny : nz);
    return pml_t(p, w) > 0 && (q < p->g.pml_lo[w] || q >= n - p->g.pml_hi[w]);
  };
  for (int c = 0; c < FD_NCLASS; ++c) {
    double acc = 0.0;
    for (const fd_tile& t : p->tiles[c])
      for (int k = t.k0; k < t.k1; ++k)
        for (int j = t.j0; j < std::min(ny, t.j0 + TY); ++j)
          for (int i = t.i0; i < std::min(nx, t.i0 + TX); ++i) {
            double b = 49.0;
            b += 32.0 * ((in_slab(0, i) ? 1 : 0) + (in_slab(1, j) ? 1 : 0) + (in_slab(2, k) ? 1 : 0));
            const uint8_t m = p->host_map[((size_t)k * ny + j) * nx + i];
            if (c >= FD_CLASS_GAIN) b += 4.0 + (p->mats[m].gain ? 84.0 : 0.0);  // ordinal and Lorentz state
            acc += b;
          }
    bytes[c] = acc;
  }
  // per DFT launch: the sample (24 bytes read, 16 written per point), and once
  // per ring the accumulators (128 bytes per point and frequency) and the ring
  double dft = 0.0;
  for (const Flux& f : p->flux)
    if (f.nf > 0) dft += (double)nx * ny * (40.0 + (128.0 * f.nf + 16.0 * FD_DFT_RING) / FD_DFT_RING);
  bytes[FD_KERNEL_DFT] = dft;
  for (int q = 0; q < 4; ++q) bytes[FD_KERNEL_DM + q] = p->dm_bytes[q];
  return FDTD_OK;
}

int fdtd_time_kernels(fdtd_plan* p, int64_t n, void* stream, double* ms, int64_t* launches) {
  if (!p || !ms || !launches) return fail(FDTD_EINVAL, "null argument");
  if (!p->bound) return fail(FDTD_ESTATE, "plan not bound");
  if (n < 0 || p->step + n > p->max_steps) return fail(FDTD_ESTATE, "max_steps exceeded");
  hipStream_t st = (hipStream_t)stream;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  auto cleanup = [&]() {
    for (Rec& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
  };
  // the events are bound to the launch itself (begin and end timestamps of the
  // kernel), so a duration excludes the gaps between launches
  auto record = [&](int cls, auto&& launch) -> int {
    Rec r{cls, nullptr, nullptr};
    HIPCHK(hipEventCreate(&r.a));
    HIPCHK(hipEventCreate(&r.b));
    recs.push_back(r);
    HIPCHK(launch(r.a, r.b));
    return FDTD_OK;
  };
  for (int64_t s = 0; s < n; ++s) {
    for (int c = 0; c < FD_NCLASS; ++c) {
      const int nt = (int)p->tiles[c].size();
      if (nt == 0) continue;
      const int grid = p->tune.max_blocks > 0 ? std::min(nt, p->tune.max_blocks) : p->pgrid[c];
      const fd_xcd* pc = p->tune.max_blocks > 0 ? nullptr : &p->part[c];
      const int r = record(c, [&](hipEvent_t a, hipEvent_t b) {
        return fd_launch_step(c, p->dtiles[c], nt, p->tune.tile_x, p->tune.block, grid, (int)s, pc, p->ntst, st, a,
                              b);
      });
      if (r) { cleanup(); return r; }
    }
    if (plan_dft_due(p, p->step + s) && !p->dft.empty()) {
      const int r = record(FD_KERNEL_DFT, [&](hipEvent_t a, hipEvent_t b) {
        return fd_launch_dft(p->ddft, (int)p->dft.size(), (int)s, st, a, b);
      });
      if (r) { cleanup(); return r; }
    }
    const DmLaunch dm = plan_dm(p);
    if (dm.n[0] > 0) {
      hipEvent_t ev[8];
      for (int q = 0; q < 4; ++q) {
        Rec r{FD_KERNEL_DM + q, nullptr, nullptr};
        if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) {
          cleanup();
          return fail(FDTD_EHIP, "time_kernels: hipEventCreate");
        }
        ev[2 * q] = r.a;
        ev[2 * q + 1] = r.b;
        if (q < 2 || dm.n[q - 1] > 0) recs.push_back(r);
        else { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); ev[2 * q] = ev[2 * q + 1] = nullptr; }
      }
      const hipError_t e = fd_launch_dm(dm.u[0], dm.n[0], dm.u[1], dm.n[1], dm.u[2], dm.n[2], p->tune.block, (int)s,
                                        st, ev);
      if (e != hipSuccess) { cleanup(); return fail(FDTD_EHIP, "time_kernels: %s", hipGetErrorString(e)); }
    }
  }
  hipError_t e = fd_launch_advance_one(p->ddesc, n, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    cleanup();
    return fail(FDTD_EHIP, "time_kernels: %s", hipGetErrorString(e));
  }
  p->step += n;
  for (int c = 0; c < FD_NKERNEL; ++c) {
    ms[c] = 0.0;
    launches[c] = 0;
  }
  for (Rec& r : recs) {
    float f = 0.0f;
    (void)hipEventElapsedTime(&f, r.a, r.b);
    ms[r.cls] += f;
    launches[r.cls] += 1;
  }
  cleanup();
  return FDTD_OK;
}

// ------------------------------------------------------------------- tuning

namespace {

// A fresh, unbound plan with p's description (grid, materials, geometry,
// sources, probes, flux planes, energy interval) and the tuning t.
fdtd_plan* clone_description(const fdtd_plan* p, const fdtd_tuning& t) {
  fdtd_plan* c = new (std::nothrow) fdtd_plan();
  if (!c) return nullptr;
  c->g = p->g;
  c->dx = p->dx;
  c->dt = p->dt;
  c->ncell = p->ncell;
  c->px = p->px;
  c->nstore = p->nstore;
  c->mats = p->mats;
  c->have_opal = p->have_opal;
  c->opal = p->opal;
  c->spheres = p->spheres;
  c->map_given = p->map_given;
  if (p->map_given) c->host_map = p->host_map;
  c->sources = p->sources;
  c->probes = p->probes;
  c->flux = p->flux;
  c->ke = p->ke;
  c->tune = t;
  return c;
}

}  // namespace

int fdtd_tune(const fdtd_plan* p, const fdtd_tuning* cand, int32_t ncand, int64_t warmup, int64_t steps,
              void* scratch, size_t bytes, size_t* need, double* ms, void* stream) {
  if (!p || !cand || ncand < 1) return fail(FDTD_EINVAL, "need a plan and at least one candidate");
  if (warmup < 0 || steps < 1 || warmup + steps > ((int64_t)1 << 31)) return fail(FDTD_EINVAL, "bad step counts");
  if (scratch && (!ms || ((uintptr_t)scratch & 255) != 0))
    return fail(FDTD_EINVAL, "timing needs ms[] and a 256-byte aligned scratch arena");
  size_t most = 0;
  for (int q = 0; q < ncand; ++q) {
    std::unique_ptr<fdtd_plan, void (*)(fdtd_plan*)> c(clone_description(p, p->tune), fdtd_plan_destroy);
    if (!c) return fail(FDTD_ENOMEM, "host allocation");
    if (fdtd_set_tuning(c.get(), &cand[q]) != FDTD_OK) {  // not a valid tuning: skipped
      if (ms) ms[q] = -1.0;
      continue;
    }
    Layout L;
    int r = compute_layout(c.get(), warmup + steps, L);
    if (r) return r;
    most = std::max(most, L.total);
    if (!scratch) continue;
    if (L.total > bytes) {
      ms[q] = -2.0;
      continue;
    }
    r = fdtd_bind_arena(c.get(), scratch, bytes, warmup + steps, stream);
    if (r) return r;
    r = plan_step(c.get(), warmup, (hipStream_t)stream);
    if (r) return r;
    double t = 0.0;
    r = fdtd_time_steps(c.get(), steps, stream, &t);
    if (r) return r;
    ms[q] = t / (double)steps;
  }
  if (need) *need = most;
  return FDTD_OK;
}

// ------------------------------------------------------------------ batches

}  // extern "C"

namespace {

// Static batches (fdtd_batch_create_static) share one table array per GPU:
// each creation takes the next generation of its device, and a batch whose
// generation is no longer the device's has lost its tables to a later one.
std::mutex g_static_mu;
uint64_t g_static_gen[FD_MAX_DEVICES] = {};

int batch_static_owner(const fdtd_batch* b) {
  if (b->static_dev < 0) return FDTD_OK;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (g_static_gen[b->static_dev] != b->static_gen)
    return fail(FDTD_ESTATE, "a later static batch on GPU %d replaced this batch's launch tables", b->static_dev);
  return FDTD_OK;
}

// Checks a member list against the batch tuning bt; *gm receives the gain model
// the members with gain share (0: none has gain).
int batch_check(fdtd_plan* const* plans, int32_t n, const fdtd_tuning& bt, int* gm) {
  if (!plans || n < 1) return fail(FDTD_EINVAL, "need at least one plan");
  for (int q = 0; q < n; ++q)
    if (!plans[q] || !plans[q]->bound) return fail(FDTD_ESTATE, "batch member %d not bound", q);
  if (bt.graph_steps < 0 || bt.max_blocks < 0 || bt.parallel < 0 || bt.parallel > 1 || bt.cache_mb < 0 ||
      bt.stores < FDTD_STORES_AUTO || bt.stores > FDTD_STORES_NONTEMPORAL)
    return fail(FDTD_EINVAL, "bad batch tuning");
  for (int q = 0; q < n; ++q) {
    if (plans[q]->tune.block != bt.block || plans[q]->tune.tile_x != bt.tile_x)
      return fail(FDTD_EINVAL, "batch members must share the block size and tile width of the batch tuning");
    for (int r = 0; r < q; ++r)
      if (plans[r] == plans[q]) return fail(FDTD_EINVAL, "plan listed twice");
  }
  *gm = 0;
  for (int q = 0; q < n; ++q) {
    if (plans[q]->gm && *gm && plans[q]->gm != *gm)
      return fail(FDTD_EUNSUPPORTED, "batch members with gain must share the gain model");
    if (plans[q]->gm) *gm = plans[q]->gm;
  }
  return FDTD_OK;
}

// Host side of a batch: members' tile lists concatenated per class, the DFT
// and density-matrix work units, and the member groups: consecutive members
// whose step state together stays within cache_mb MB (a member larger than
// that is a group of its own; cache_mb = 0: one group), each with the XCD
// partitions of its own tiles.
void batch_layout(fdtd_batch* b, fdtd_plan* const* plans, int32_t n, int gm) {
  b->plans.assign(plans, plans + n);
  b->gm = gm ? gm : 1;
  b->maxnf = 0;
  b->dft.clear();
  b->groups.clear();
  for (int c = 0; c < FD_NCLASS; ++c) b->tiles[c].clear();
  for (int q = 0; q < 3; ++q) b->dmu[q].clear();
  const size_t cap = (size_t)b->cache_mb << 20;
  size_t held = 0;
  std::vector<double> gcost[FD_NCLASS];
  auto close_group = [&]() {
    BGroup& g = b->groups.back();
    for (int c = 0; c < FD_NCLASS; ++c) {
      g.nt[c] = (int)b->tiles[c].size() - g.t0[c];
      g.part[c] = xcd_partition(gcost[c], &g.pgrid[c]);
      gcost[c].clear();
    }
    g.nd = (int)b->dft.size() - g.d0;
    for (int q = 0; q < 3; ++q) g.nu[q] = (int)b->dmu[q].size() - g.u0[q];
  };
  for (int m = 0; m < n; ++m) {
    fdtd_plan* p = b->plans[m];
    const size_t bytes = step_state_bytes(p);
    if (b->groups.empty() || (cap > 0 && held > 0 && held + bytes > cap)) {
      if (!b->groups.empty()) close_group();
      BGroup g;
      g.m0 = m;
      for (int c = 0; c < FD_NCLASS; ++c) g.t0[c] = (int)b->tiles[c].size();
      g.d0 = (int)b->dft.size();
      for (int q = 0; q < 3; ++q) g.u0[q] = (int)b->dmu[q].size();
      b->groups.push_back(g);
      held = 0;
    }
    BGroup& g = b->groups.back();
    g.m1 = m + 1;
    g.maxnf = std::max(g.maxnf, p->maxnf);
    held += bytes;
    for (int c = 0; c < FD_NCLASS; ++c) {
      b->tiles[c].insert(b->tiles[c].end(), p->tiles[c].begin(), p->tiles[c].end());
      gcost[c].insert(gcost[c].end(), p->tcost[c].begin(), p->tcost[c].end());
    }
    b->dft.insert(b->dft.end(), p->dft.begin(), p->dft.end());
    b->maxnf = std::max(b->maxnf, p->maxnf);
    for (int q = 0; q < 3; ++q) b->dmu[q].insert(b->dmu[q].end(), p->dmu[q].begin(), p->dmu[q].end());
  }
  close_group();
}

// Device bytes of the batch's launch tables (tile lists, DFT units, descriptor
// pointers) and their offsets.
size_t batch_table_bytes(const fdtd_batch* b, size_t off_t[FD_NCLASS], size_t* off_d, size_t* off_p,
                         size_t off_m[3]) {
  size_t bytes = 0;
  for (int c = 0; c < FD_NCLASS; ++c) {
    off_t[c] = bytes;
    bytes = align256(bytes + sizeof(fd_tile) * b->tiles[c].size());
  }
  *off_d = bytes;
  bytes = align256(bytes + sizeof(fd_dft_tile) * std::max<size_t>(b->dft.size(), 1));
  for (int q = 0; q < 3; ++q) {
    off_m[q] = bytes;
    bytes = align256(bytes + sizeof(fd_dm_unit) * b->dmu[q].size());
  }
  *off_p = bytes;
  return align256(bytes + sizeof(fd_desc*) * b->plans.size());
}

void batch_drop_graphs(fdtd_batch* b) {
  for (auto& kv : b->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  b->graphs.clear();
}

// Writes the launch tables of b's members to b->dmem (b->dcap bytes, the
// caller has checked they fit) and points the launch arguments at them.
int batch_upload(fdtd_batch* b) {
  size_t off_t[FD_NCLASS], off_d, off_p, off_m[3];
  (void)batch_table_bytes(b, off_t, &off_d, &off_p, off_m);
  uint8_t* base = (uint8_t*)b->dmem;
  std::vector<fd_desc*> dl;
  for (fdtd_plan* p : b->plans) dl.push_back(p->ddesc);
  for (int c = 0; c < FD_NCLASS; ++c) {
    b->dtiles[c] = (fd_tile*)(base + off_t[c]);
    if (!b->tiles[c].empty())
      HIPCHK(hipMemcpy(b->dtiles[c], b->tiles[c].data(), sizeof(fd_tile) * b->tiles[c].size(), hipMemcpyHostToDevice));
  }
  b->ddft = (fd_dft_tile*)(base + off_d);
  if (!b->dft.empty())
    HIPCHK(hipMemcpy(b->ddft, b->dft.data(), sizeof(fd_dft_tile) * b->dft.size(), hipMemcpyHostToDevice));
  for (int q = 0; q < 3; ++q) {
    b->ddm[q] = (fd_dm_unit*)(base + off_m[q]);
    if (!b->dmu[q].empty())
      HIPCHK(hipMemcpy(b->ddm[q], b->dmu[q].data(), sizeof(fd_dm_unit) * b->dmu[q].size(), hipMemcpyHostToDevice));
  }
  b->ddescs = (fd_desc**)(base + off_p);
  HIPCHK(hipMemcpy(b->ddescs, dl.data(), sizeof(fd_desc*) * dl.size(), hipMemcpyHostToDevice));
  return FDTD_OK;
}

}  // namespace

extern "C" {

int fdtd_batch_create(fdtd_plan* const* plans, int32_t n, const fdtd_tuning* t, fdtd_batch** out) {
  if (!plans || !out || n < 1) return fail(FDTD_EINVAL, "need at least one plan");
  *out = nullptr;
  if (!plans[0]) return fail(FDTD_ESTATE, "batch member 0 not bound");
  const fdtd_tuning bt = t ? *t : plans[0]->tune;
  int gm = 0;
  if (int r = batch_check(plans, n, bt, &gm)) return r;
  std::unique_ptr<fdtd_batch> b(new (std::nothrow) fdtd_batch());
  if (!b) return fail(FDTD_ENOMEM, "host allocation");
  b->block = bt.block;
  b->tile_x = bt.tile_x;
  b->parallel = bt.parallel;
  b->max_blocks = bt.max_blocks;
  b->graph_steps = bt.graph_steps;
  b->cache_mb = bt.cache_mb;
  // Batches keep ordinary stores unless asked: over a 64-member ensemble of
  // 1.9 GB the non-temporal form measured about 10% slower, while a single 2 GB
  // grid gains.
  b->ntst = bt.stores == FDTD_STORES_NONTEMPORAL ? 1 : 0;
  batch_layout(b.get(), plans, n, gm);
  size_t off_t[FD_NCLASS], off_d, off_p, off_m[3];
  const size_t bytes = batch_table_bytes(b.get(), off_t, &off_d, &off_p, off_m);
  // Set-up allocation of the batch's launch tables (small; grown by
  // fdtd_batch_set_members only when a member list needs more; freed by destroy).
  HIPCHK(hipMalloc(&b->dmem, bytes));
  b->dcap = bytes;
  b->owns_dmem = true;
  if (int r = batch_upload(b.get())) {
    (void)hipFree(b->dmem);
    b->dmem = nullptr;
    return r;
  }
  *out = b.release();
  return FDTD_OK;
}

int fdtd_batch_create_static(fdtd_plan* const* plans, int32_t n, const fdtd_tuning* t, fdtd_batch** out) {
  if (!plans || !out || n < 1) return fail(FDTD_EINVAL, "need at least one plan");
  *out = nullptr;
  if (!plans[0]) return fail(FDTD_ESTATE, "batch member 0 not bound");
  const fdtd_tuning bt = t ? *t : plans[0]->tune;
  int gm = 0;
  if (int r = batch_check(plans, n, bt, &gm)) return r;
  std::unique_ptr<fdtd_batch> b(new (std::nothrow) fdtd_batch());
  if (!b) return fail(FDTD_ENOMEM, "host allocation");
  b->block = bt.block;
  b->tile_x = bt.tile_x;
  b->parallel = bt.parallel;
  b->max_blocks = bt.max_blocks;
  b->graph_steps = bt.graph_steps;
  b->cache_mb = bt.cache_mb;
  b->ntst = bt.stores == FDTD_STORES_NONTEMPORAL ? 1 : 0;
  batch_layout(b.get(), plans, n, gm);
  size_t off_t[FD_NCLASS], off_d, off_p, off_m[3];
  const size_t bytes = batch_table_bytes(b.get(), off_t, &off_d, &off_p, off_m);
  if (bytes > FD_STATIC_TABLE_BYTES)
    return fail(FDTD_ENOMEM, "batch launch tables of %zu bytes exceed the static maximum of %zu", bytes,
                (size_t)FD_STATIC_TABLE_BYTES);
  void* base = nullptr;
  int dev = 0;
  HIPCHK(fd_static_tables(&base, &dev));
  b->dmem = base;
  b->dcap = FD_STATIC_TABLE_BYTES;
  b->owns_dmem = false;
  b->static_dev = dev;
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    b->static_gen = ++g_static_gen[dev];
  }
  if (int r = batch_upload(b.get())) return r;
  *out = b.release();
  return FDTD_OK;
}

int fdtd_batch_set_members(fdtd_batch* b, fdtd_plan* const* plans, int32_t n, void* stream) {
  if (!b) return fail(FDTD_EINVAL, "null batch");
  if (int r = batch_static_owner(b)) return r;
  fdtd_tuning bt{};
  bt.block = b->block;
  bt.tile_x = b->tile_x;
  bt.graph_steps = b->graph_steps;
  bt.max_blocks = b->max_blocks;
  bt.parallel = b->parallel;
  bt.stores = b->ntst ? FDTD_STORES_NONTEMPORAL : FDTD_STORES_ORDINARY;
  bt.cache_mb = b->cache_mb;
  int gm = 0;
  if (int r = batch_check(plans, n, bt, &gm)) return r;
  // the launches already queued read the current tables: wait for them
  HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  fdtd_batch next;
  next.cache_mb = b->cache_mb;
  batch_layout(&next, plans, n, gm);
  size_t off_t[FD_NCLASS], off_d, off_p, off_m[3];
  const size_t bytes = batch_table_bytes(&next, off_t, &off_d, &off_p, off_m);
  if (bytes > b->dcap) {
    if (!b->owns_dmem) return fail(FDTD_ENOMEM, "member tables of %zu bytes exceed the %zu available", bytes, b->dcap);
    void* grown = nullptr;
    HIPCHK(hipMalloc(&grown, bytes + bytes / 2));
    (void)hipFree(b->dmem);
    b->dmem = grown;
    b->dcap = bytes + bytes / 2;
  }
  batch_drop_graphs(b);
  batch_layout(b, plans, n, gm);
  return batch_upload(b);
}

void fdtd_batch_destroy(fdtd_batch* b) {
  if (!b) return;
  batch_drop_graphs(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->dmem && b->owns_dmem) (void)hipFree(b->dmem);
  delete b;
}

static bool group_dft_due(const fdtd_batch* b, const BGroup& g, int64_t s) {
  for (int m = g.m0; m < g.m1; ++m)
    if (plan_dft_due(b->plans[m], b->plans[m]->step + s)) return true;
  return false;
}

static DmLaunch group_dm(const fdtd_batch* b, const BGroup& g) {
  DmLaunch l;
  for (int q = 0; q < 3; ++q) {
    l.u[q] = b->ddm[q] + g.u0[q];
    l.n[q] = g.nu[q];
  }
  return l;
}

// n steps of every member, group after group (a group's state stays in the
// Infinity Cache over its n steps when it fits there); members are independent,
// so the order changes no result.
static int batch_enqueue(fdtd_batch* b, int64_t n, hipStream_t st, Fork* fk) {
  for (const BGroup& g : b->groups) {
    fd_tile* dt[FD_NCLASS];
    for (int c = 0; c < FD_NCLASS; ++c) dt[c] = b->dtiles[c] + g.t0[c];
    const DmLaunch dm = group_dm(b, g);
    for (int64_t s = 0; s < n; ++s) {
      const int r = enqueue_step(dt, g.nt, g.part, g.pgrid, b->tile_x, b->block, b->max_blocks, b->ddft + g.d0, g.nd,
                                 g.maxnf, group_dft_due(b, g, s), (int)s, b->ntst, dm, st, fk);
      if (r) return r;
    }
  }
  HIPCHK(fd_launch_advance(b->ddescs, (int)b->plans.size(), n, st));
  return FDTD_OK;
}

static int batch_step(fdtd_batch* b, int64_t n, hipStream_t st) {
  if (n < 0) return fail(FDTD_EINVAL, "negative step count");
  if (int r = batch_static_owner(b)) return r;
  for (fdtd_plan* p : b->plans)
    if (p->step + n > p->max_steps) return fail(FDTD_ESTATE, "a member would exceed its max_steps");
  const int64_t K = b->graph_steps;
  int64_t done = 0;
  if (K > 0) {
    while (n - done >= K) {
      std::vector<int64_t> key{K};
      for (fdtd_plan* p : b->plans) key.push_back(plan_phase_key(p, p->step));
      auto it = b->graphs.find(key);
      if (it == b->graphs.end()) {
        if (!b->cap) HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        Fork* fk = nullptr;
        if (b->parallel) {
          if (!b->fork) b->fork.reset(new Fork());
          if (int rf = b->fork->init()) return rf;
          fk = b->fork.get();
        }
        GraphEntry ge;
        HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        const int r = batch_enqueue(b, K, b->cap, fk);
        hipGraph_t gr = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap, &gr);
        if (r) {
          if (gr) (void)hipGraphDestroy(gr);
          return r;
        }
        if (e != hipSuccess) return fail(FDTD_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        ge.graph = gr;
        HIPCHK(hipGraphInstantiate(&ge.exec, gr, nullptr, nullptr, 0));
        it = b->graphs.emplace(key, ge).first;
      }
      HIPCHK(hipGraphLaunch(it->second.exec, st));
      for (fdtd_plan* p : b->plans) p->step += K;
      done += K;
    }
  }
  if (n - done > 0) {
    const int r = batch_enqueue(b, n - done, st, nullptr);
    if (r) return r;
    for (fdtd_plan* p : b->plans) p->step += n - done;
  }
  return FDTD_OK;
}

int fdtd_batch_step(fdtd_batch* b, int64_t n, void* stream) {
  if (!b) return fail(FDTD_EINVAL, "null batch");
  return batch_step(b, n, (hipStream_t)stream);
}

int fdtd_batch_time_kernels(fdtd_batch* b, int64_t n, void* stream, double* ms, int64_t* launches) {
  if (!b || !ms || !launches) return fail(FDTD_EINVAL, "null argument");
  if (n < 0) return fail(FDTD_EINVAL, "negative step count");
  if (int r = batch_static_owner(b)) return r;
  for (fdtd_plan* p : b->plans)
    if (p->step + n > p->max_steps) return fail(FDTD_ESTATE, "a member would exceed its max_steps");
  hipStream_t st = (hipStream_t)stream;
  std::vector<std::array<hipEvent_t, 2>> ev;
  std::vector<int> cls;
  std::set<std::pair<int, int64_t>> stepped;  // (kernel, step) pairs launched
  int64_t cur = 0;
  auto cleanup = [&]() {
    for (auto& e : ev) {
      (void)hipEventDestroy(e[0]);
      (void)hipEventDestroy(e[1]);
    }
  };
  auto pair = [&](int c, hipEvent_t* a, hipEvent_t* z) -> int {
    std::array<hipEvent_t, 2> e{};
    HIPCHK(hipEventCreate(&e[0]));
    HIPCHK(hipEventCreate(&e[1]));
    ev.push_back(e);
    cls.push_back(c);
    stepped.insert({c, cur});
    *a = e[0];
    *z = e[1];
    return FDTD_OK;
  };
  for (const BGroup& g : b->groups)
  for (int64_t s = 0; s < n; ++s) {
    cur = s;
    for (int c = 0; c < FD_NCLASS; ++c) {
      const int nt = g.nt[c];
      if (nt == 0) continue;
      const int grid = b->max_blocks > 0 ? std::min(nt, b->max_blocks) : g.pgrid[c];
      const fd_xcd* pc = b->max_blocks > 0 ? nullptr : &g.part[c];
      hipEvent_t a, z;
      if (int r = pair(c, &a, &z)) { cleanup(); return r; }
      const hipError_t e = fd_launch_step(c, b->dtiles[c] + g.t0[c], nt, b->tile_x, b->block, grid, (int)s, pc,
                                          b->ntst, st, a, z);
      if (e != hipSuccess) { cleanup(); return fail(FDTD_EHIP, "batch_time_kernels: %s", hipGetErrorString(e)); }
    }
    if (group_dft_due(b, g, s) && g.nd > 0) {
      hipEvent_t a, z;
      if (int r = pair(FD_KERNEL_DFT, &a, &z)) { cleanup(); return r; }
      const hipError_t e = fd_launch_dft(b->ddft + g.d0, g.nd, (int)s, st, a, z);
      if (e != hipSuccess) { cleanup(); return fail(FDTD_EHIP, "batch_time_kernels: %s", hipGetErrorString(e)); }
    }
    const DmLaunch dm = group_dm(b, g);
    if (dm.n[0] > 0) {
      hipEvent_t ev[8] = {};
      for (int q = 0; q < 4; ++q)
        if (q < 2 || dm.n[q - 1] > 0)
          if (int r = pair(FD_KERNEL_DM + q, &ev[2 * q], &ev[2 * q + 1])) { cleanup(); return r; }
      const hipError_t e = fd_launch_dm(dm.u[0], dm.n[0], dm.u[1], dm.n[1], dm.u[2], dm.n[2], b->block, (int)s, st,
                                        ev);
      if (e != hipSuccess) { cleanup(); return fail(FDTD_EHIP, "batch_time_kernels: %s", hipGetErrorString(e)); }
    }
  }
  hipError_t e = fd_launch_advance(b->ddescs, (int)b->plans.size(), n, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    cleanup();
    return fail(FDTD_EHIP, "batch_time_kernels: %s", hipGetErrorString(e));
  }
  for (fdtd_plan* p : b->plans) p->step += n;
  for (int c = 0; c < FD_NKERNEL; ++c) {
    ms[c] = 0.0;
    launches[c] = 0;
  }
  for (size_t q = 0; q < ev.size(); ++q) {
    float f = 0.0f;
    (void)hipEventElapsedTime(&f, ev[q][0], ev[q][1]);
    ms[cls[q]] += f;
  }
  for (const auto& cs : stepped) launches[cs.first] += 1;
  cleanup();
  return FDTD_OK;
}

int fdtd_batch_time_steps(fdtd_batch* b, int64_t n, void* stream, double* ms) {
  if (!b || !ms) return fail(FDTD_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, st));
  const int r = batch_step(b, n, st);
  if (r) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r;
  }
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(hipEventSynchronize(e1));
  float f = 0.0f;
  HIPCHK(hipEventElapsedTime(&f, e0, e1));
  *ms = f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return FDTD_OK;
}

}  // extern "C"
