// gfx950 kernels of libfdtd: one fused Yee step (H then E, CPML, the Lorentz
// gain medium -- ADE with four-level populations and noise -- soft sources,
// probes, transmitted power, energy), the passes of the density-matrix gain
// medium (a ground level and three degenerate upper levels, held at the cell
// centre), the running-DFT flux update, the integer voxelizer and small helpers.
//
// Method: C. Conti and A. Fratalocchi, arXiv:0802.3775 — Yee FDTD with absorbing
// walls in a disordered inverted opal, pumped gain medium seeded by a stochastic
// source, transmitted power T(t) (sections "Sample and numerical approach" and
// "Dynamical diffusion and localization").
//
// Stepping scheme.  E, H, the H-side CPML memory and the Lorentz polarization
// are double-buffered by step parity, so one step reads only buffer n&1 and
// writes only the other one (the E-side CPML memory and the populations are read
// and written only by their own cell's thread).  Every tile is therefore
// independent within a step, and a
// workgroup can recompute the H^{n+1/2} values its E update needs at x-1, y-1 and
// z-1 from the read-only inputs instead of waiting for the owner: one pass over
// HBM per step (E, H, material index in; E, H out).
//
// Work mapping.  A tile is `block` consecutive (i,j) columns of the flattened xy
// plane (x fastest, so every wavefront reads 64 contiguous floats per array) and a
// z range [k0, k1) that the workgroup marches upward, carrying the H^{n+1/2} of
// plane k-1 in registers.  Tiles whose columns touch no CPML slab and no gain cell
// run a specialised kernel without that code.
#include "fd_internal.h"

#include <hip/hip_ext.h>

#include <mutex>
#include <type_traits>

namespace {

constexpr float kTwoPiF = 6.28318530717958647692f;

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c[0];
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t y0 = hi1 ^ c[1] ^ k0;
    const uint32_t y2 = hi0 ^ c[3] ^ k1;
    c[0] = y0; c[1] = lo1; c[2] = y2; c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ float u24(uint32_t x) {
  return (static_cast<float>(x >> 8) + 0.5f) * 5.9604644775390625e-8f;  // 2^-24
}

// Three standard normals for (step n, cell o): Box-Muller on the uniform pairs.
__device__ __forceinline__ void normals3(uint32_t n, uint32_t o, uint32_t k0, uint32_t k1, float g[3]) {
  uint32_t c[4] = {n, o, 0u, 2u};
  philox10(c, k0, k1);
  const float r0 = sqrtf(-2.0f * logf(u24(c[0])));
  float s0, c0;
  sincosf(kTwoPiF * u24(c[1]), &s0, &c0);
  const float r1 = sqrtf(-2.0f * logf(u24(c[2])));
  g[0] = r0 * c0;
  g[1] = r0 * s0;
  g[2] = r1 * cosf(kTwoPiF * u24(c[3]));
}

// ------------------------------------------------------------------ context
// Field arrays are reached through pointers stored in the plan's descriptor, so
// the compiler cannot infer their address space; every pointer is cast to the
// global space (1) so loads and stores are global_* instructions, and the
// descriptor itself to the constant space (4) so its fields are scalar loads.
typedef __attribute__((address_space(1))) float gf;
typedef __attribute__((address_space(1))) double gd;
typedef __attribute__((address_space(1))) uint8_t gu8;
typedef __attribute__((address_space(4))) fd_desc cdesc;
typedef __attribute__((address_space(4))) fd_mat cmat;
typedef __attribute__((address_space(4))) const float cfloat;

__device__ __forceinline__ gf* G(float* p) { return (gf*)p; }
__device__ __forceinline__ const gf* G(const float* p) { return (const gf*)p; }
__device__ __forceinline__ gd* G(double* p) { return (gd*)p; }
__device__ __forceinline__ const gd* G(const double* p) { return (const gd*)p; }

// A field array indexed with a 32-bit element index: the byte offset is formed
// in 32 bits and zero-extended, so loads and stores take the scalar-base +
// 32-bit vector-offset form (one VGPR per address, no 64-bit address adds).
// Valid for arrays below 4 GiB, which every per-cell array is (at most 2^30
// cells of 4 bytes).
typedef __attribute__((address_space(1))) char gchar;
typedef __attribute__((address_space(1))) const char gcchar;
template <class T>
struct R32 {
  __attribute__((address_space(1))) T* p;
  __device__ __forceinline__ __attribute__((address_space(1))) T& operator[](uint32_t i) const {
    typedef __attribute__((address_space(1))) T gT;
    typedef typename std::conditional<std::is_const<T>::value, gcchar, gchar>::type gb;
    return *(gT*)((gb*)p + (size_t)(i * (uint32_t)sizeof(T)));
  }
};

struct Ctx {
  int nx, ny, nz, plane;
  int rx;  // row pitch of the per-cell arrays
  int px, py, pz;
  float ch;
  R32<const float> Ein[3];
  R32<float> Eout[3];
  R32<const float> Hin[3];
  R32<float> Hout[3];
  // CPML (used by the kernels specialised with PML)
  int lo[3], hi[3], t[3], n[3];
  const cfloat* prof[3];  // read-only for the kernel: scalar loads where uniform
  R32<float> psiE[3][2];
  R32<const float> psiHin[3][2];
  R32<float> psiHout[3][2];
};

__device__ __forceinline__ void make_ctx(Ctx& x, const cdesc* d, int par, bool pml) {
  x.nx = d->nx; x.ny = d->ny; x.nz = d->nz; x.plane = d->plane; x.rx = d->px;
  x.px = d->per[0]; x.py = d->per[1]; x.pz = d->per[2];
  x.ch = d->ch;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    x.Ein[c].p = G((const float*)d->E[par][c]);
    x.Eout[c].p = G(d->E[par ^ 1][c]);
    x.Hin[c].p = G((const float*)d->H[par][c]);
    x.Hout[c].p = G(d->H[par ^ 1][c]);
  }
  x.n[0] = d->nx; x.n[1] = d->ny; x.n[2] = d->nz;
  if (!pml) return;
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    x.lo[w] = d->pml_lo[w]; x.hi[w] = d->pml_hi[w]; x.t[w] = d->pml_t[w];
    x.prof[w] = (const cfloat*)d->prof[w];
    // an axis without CPML has no psi arrays: its pointers are set to E so
    // that the unconditional reads of the all-axes march stay in bounds (their
    // values are never used; stores happen only inside slabs)
    float* const spare = d->E[par][0];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      x.psiE[w][f].p = G(d->psiE[w][f] ? d->psiE[w][f] : spare);
      x.psiHin[w][f].p = G((const float*)(d->psiH[par][w][f] ? d->psiH[par][w][f] : spare));
      x.psiHout[w][f].p = G(d->psiH[par ^ 1][w][f] ? d->psiH[par ^ 1][w][f] : spare);
    }
  }
}

__device__ __forceinline__ int nxt(int i, int n, int per) { return i + 1 < n ? i + 1 : (per ? 0 : -1); }
__device__ __forceinline__ int prv(int i, int n, int per) { return i > 0 ? i - 1 : (per ? n - 1 : -1); }

// index along an axis after periodic wrap, or -1 beyond a PEC wall
__device__ __forceinline__ int wrap(int i, int n, int per) {
  if (i >= 0 && i < n) return i;
  if (!per) return -1;
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// slab-local index along axis w, or -1 outside the slabs
__device__ __forceinline__ int slab(const Ctx& x, int w, int p) {
  if (x.t[w] == 0) return -1;
  if (p < x.lo[w]) return p;
  if (p >= x.n[w] - x.hi[w]) return p - (x.n[w] - x.hi[w]) + x.lo[w];
  return -1;
}

// psi array offset for axis w, slab index sp, at (i, j, k)
__device__ __forceinline__ int psi_off(const Ctx& x, int w, int sp, int i, int j, int k) {
  if (w == 2) return sp * x.plane + j * x.rx + i;
  if (w == 0) return (k * x.ny + j) * x.t[0] + sp;
  return (k * x.t[1] + sp) * x.nx + i;
}

// family of component c within axis w's two stored psi arrays
__device__ __forceinline__ int fam(int c, int w) { return c == (w + 1) % 3 ? 0 : 1; }

// CPML stretch of one difference d along axis w at index p (E position when
// HSIDE = false, H position when HSIDE = true): returns d/kappa + psi with the
// psi recursion psi = b psi + c d; the owner of the cell stores psi.
template <bool HSIDE, int PM>
__device__ __forceinline__ float stretch(const Ctx& x, int c, int w, int p, int i, int j, int k, float d,
                                         bool own) {
  if (!((PM >> w) & 1)) return d;  // no slab on this axis in this tile class
  const int sp = slab(x, w, p);
  if (sp < 0) return d;
  const cfloat* pr = x.prof[w] + (HSIDE ? 3 : 0) * x.n[w];
  const float kinv = pr[p], b = pr[x.n[w] + p], cc = pr[2 * x.n[w] + p];
  const int off = psi_off(x, w, sp, i, j, k);
  const int f = fam(c, w);
  float psi;
  if (HSIDE) {
    psi = fmaf(b, x.psiHin[w][f][off], cc * d);
    if (own) x.psiHout[w][f][off] = psi;
  } else {
    psi = fmaf(b, x.psiE[w][f][off], cc * d);
    if (own) x.psiE[w][f][off] = psi;
  }
  return fmaf(d, kinv, psi);
}

// The same for a z difference when the old psi and the plane's grading
// (pz = 1/kappa, b, c) have already been loaded: z slabs are whole planes, so
// the slab index sz of plane k is uniform over a tile.  off2d: j*px + i of the
// cell.  Bit-identical to stretch<HSIDE, PM>(.., 2, k, ..).
template <bool HSIDE>
__device__ __forceinline__ float stretch_z(const Ctx& x, int c, const float* pz, int sz, int off2d, float d,
                                           bool own, float psi_old) {
  if (sz < 0) return d;
  const float kinv = pz[0], b = pz[1], cc = pz[2];
  const float psi = fmaf(b, psi_old, cc * d);
  if (own) {
    const int off = sz * x.plane + off2d;
    if (HSIDE) x.psiHout[2][fam(c, 2)][off] = psi;
    else x.psiE[2][fam(c, 2)][off] = psi;
  }
  return fmaf(d, kinv, psi);
}

// A CPML difference whose old psi and grading are already in registers (sp: slab
// index, -1 outside): returns d/kappa + psi with psi = b psi_old + c d and stores
// psi at dst[off] when own.  Bit-identical to stretch<HSIDE, PM>.
__device__ __forceinline__ float stretch_v(float d, int sp, float kinv, float b, float cc, float psi_old, bool own,
                                           const R32<float>& dst, uint32_t off) {
  if (sp < 0) return d;
  const float psi = fmaf(b, psi_old, cc * d);
  if (own) dst[off] = psi;
  return fmaf(d, kinv, psi);
}

// One H component from its two differences: H^{n+1/2} = H^{n-1/2} - (dt/dx)(d1 - d2),
// each difference stretched by the CPML where the position lies in a slab.  The
// owner and every workgroup that recomputes the value as a halo call this with
// identical operands, so all copies agree bit for bit.
// c: component; (w1, p1) / (w2, p2): axis and index of the two differences.
// ZPRE: a z difference takes its old psi from zpsi (slab index sz, cell off2d).
template <int PM, bool ZPRE = false>
__device__ __forceinline__ float h_from(const Ctx& x, int c, int w1, int p1, int w2, int p2, int i, int j, int k,
                                        float a1, float a0, float b1, float b0, float hold, bool own, int sz = -1,
                                        int off2d = 0, float zpsi = 0.0f, const float* pz = nullptr) {
  float d1 = a1 - a0, d2 = b1 - b0;
  if (PM) {
    d1 = (ZPRE && w1 == 2) ? stretch_z<true>(x, c, pz, sz, off2d, d1, own, zpsi)
                           : stretch<true, PM>(x, c, w1, p1, i, j, k, d1, own);
    d2 = (ZPRE && w2 == 2) ? stretch_z<true>(x, c, pz, sz, off2d, d2, own, zpsi)
                           : stretch<true, PM>(x, c, w2, p2, i, j, k, d2, own);
  }
  return fmaf(-x.ch, d1 - d2, hold);
}

// The H-side stretch of a difference of the plane below a tile (the prologue
// of the all-axes march; no psi store), in two parts so that the loads go out
// with the prologue's other loads, whatever the lane's slab membership (index 0
// outside a slab; the result is selected): pre_load issues them, pre_apply is
// stretch<true, PM>(.., own = false) bit for bit.
struct PreStretch {
  float kinv, b, cc, po;
  bool in;
};
template <int PM>
__device__ __forceinline__ PreStretch pre_load(const Ctx& x, int c, int w, int p, int i, int j, int k, bool live) {
  PreStretch r{1.0f, 0.0f, 0.0f, 0.0f, false};
  if (!((PM >> w) & 1) || x.t[w] == 0) return r;  // uniform: no slab code on this axis
  const int sp = slab(x, w, p);
  r.in = live && sp >= 0;
  const cfloat* pr = x.prof[w] + 3 * x.n[w];
  const int pc = r.in ? p : 0;
  r.kinv = pr[pc];
  r.b = pr[x.n[w] + pc];
  r.cc = pr[2 * x.n[w] + pc];
  r.po = x.psiHin[w][fam(c, w)][r.in ? psi_off(x, w, sp, i, j, k) : 0];
  return r;
}
__device__ __forceinline__ float pre_apply(const PreStretch& r, float d) {
  const float psi = fmaf(r.b, r.po, r.cc * d);
  return r.in ? fmaf(d, r.kinv, psi) : d;
}

// Workgroup barrier for LDS traffic only.  Within a step no workgroup reads
// global memory that another thread of the step writes (inputs and outputs are
// separate buffers), so the barrier waits for outstanding LDS operations but
// not for global loads in flight: loads issued for the next z-plane keep
// streaming across it.
__device__ __forceinline__ void lds_barrier() {
  __asm__ __volatile__("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Deterministic block sum (fixed shuffle tree, then wave partials in order).
__device__ double block_sum(double v, double* sred) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  lds_barrier();
  if (lane == 0) sred[w] = v;
  lds_barrier();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) r += sred[q];
  return r;
}

// (hi, lo) += inc as an unevaluated FP32 pair (Knuth's two-sum, then renormalise).
__device__ __forceinline__ void two_sum(float& hi, float& lo, float inc) {
  const float s = hi + inc;
  const float bb = s - hi;
  const float err = (hi - (s - bb)) + (inc - bb);
  const float l = lo + err;
  const float h2 = s + l;
  lo = l - (h2 - s);
  hi = h2;
}

// ------------------------------------------------- density-matrix gain cells
// State of one cell in registers: upper-level populations rho_kk as (hi, lo)
// pairs, the ground-upper coherences rho_0k = cr + i ci and the upper-upper
// coherences rho_12, rho_13, rho_23 = xr + i xi.  The trace is fixed at 1, so
// rho_00 = 1 - sum rho_kk (the real su(4) coordinates of the paper's model,
// with the diagonal held as level populations).
struct Cz {
  float r, i;
};
__device__ __forceinline__ Cz zm(Cz a, Cz b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ Cz zc(Cz a) { return {a.r, -a.i}; }
__device__ __forceinline__ Cz za(Cz a, Cz b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ Cz zs(Cz a, float s) { return {a.r * s, a.i * s}; }

// Half-step relaxation R(dt/2): exact flow of T1 decay, pump and T2 dephasing.
// p: populations (updated), inc: their accumulated increments.
__device__ __forceinline__ void dm_relax(const fd_mat& mt, float p[3], float inc[3], Cz c[3], Cz x[3]) {
  const float e = (p[0] + p[1]) + p[2];
  const float de3 = (mt.beinf - e) * mt.bg1m * (1.0f / 3.0f);
  const float e3 = e * (1.0f / 3.0f);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float d = de3 - (p[k] - e3) * mt.bh1m;
    inc[k] += d;
    p[k] += d;
    c[k] = zs(c[k], mt.bf2);
    x[k] = zs(x[k], mt.bf2);
  }
}

// Cayley step C(E): rho -> V rho V^+, V = (I + i tau H')^{-1}(I - i tau H'),
// tau = dt/2.  In closed form (D = 1 + tau^2 |E|^2 + i w' tau):
//   V_00 = (1 + i w' tau - tau^2 |E|^2) / D,  V_0k = V_k0 = 2 i tau E_k / D,
//   V_kl = r delta_kl + g E_k E_l,  r = (1 - i w' tau)/(1 + i w' tau),
//   g = -2 tau^2 / (D (1 + i w' tau)).
// With w_k = rho_k0, y = X^T E (X the upper block), s = E.w, q = E.X.E:
//   T_k0 = E_k (b p00 + g s) + r w_k,  z_k = E_k (b s* + g q) + r y_k*,
//   rho'_k0 = a* T_k0 + b* z_k,
//   rho'_kl = X_kl + r* E_k (b w_l* + g y_l) + E_l (b* T_k0 + g* z_k)
// (a = V_00, b = V_0k / E_k).  FULL = false stops after rho'_k0 (the predictor).
template <bool FULL>
__device__ __forceinline__ void dm_cayley(const fd_mat& mt, const float E[3], float p[3], float inc[3], Cz c[3],
                                          Cz x[3]) {
  const float tau = mt.btau;
  const float t2e = tau * tau * fmaf(E[0], E[0], fmaf(E[1], E[1], E[2] * E[2]));
  const float dr = 1.0f + t2e, di = mt.bwt;
  const float inv = 1.0f / fmaf(dr, dr, di * di);
  const Cz iD = {dr * inv, -di * inv};
  const Cz al = zm({1.0f - t2e, di}, iD);
  const Cz be = {-2.0f * tau * iD.i, 2.0f * tau * iD.r};
  const Cz ga = zs(zm(iD, {mt.bc1r, mt.bc1i}), -2.0f * tau * tau);
  const Cz rr = {mt.brr, mt.bri};
  const float p00 = 1.0f - ((p[0] + p[1]) + p[2]);
  Cz w[3], y[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) w[k] = zc(c[k]);
  // upper block: X_kk = p_k, X_01 = x0, X_02 = x1, X_12 = x2, X_lk = X_kl*
  y[0] = za(za({E[0] * p[0], 0.0f}, zs(zc(x[0]), E[1])), zs(zc(x[1]), E[2]));
  y[1] = za(za(zs(x[0], E[0]), {E[1] * p[1], 0.0f}), zs(zc(x[2]), E[2]));
  y[2] = za(za(zs(x[1], E[0]), zs(x[2], E[1])), {E[2] * p[2], 0.0f});
  const Cz sv = za(za(zs(w[0], E[0]), zs(w[1], E[1])), zs(w[2], E[2]));
  const float qv = fmaf(E[0], y[0].r, fmaf(E[1], y[1].r, E[2] * y[2].r));
  const Cz u0 = za(zs(be, p00), zm(ga, sv));
  const Cz u1 = za(zm(be, zc(sv)), zs(ga, qv));
  Cz T[3], z[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T[k] = za(zs(u0, E[k]), zm(rr, w[k]));
    z[k] = za(zs(u1, E[k]), zm(rr, zc(y[k])));
    c[k] = zc(za(zm(zc(al), T[k]), zm(zc(be), z[k])));  // rho'_0k = (rho'_k0)*
  }
  if (!FULL) return;
  Cz a[3], b[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a[k] = zm(zc(rr), za(zm(be, zc(w[k])), zm(ga, y[k])));  // r* (b w_k* + g y_k)
    b[k] = za(zm(zc(be), T[k]), zm(zc(ga), z[k]));
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float d = E[k] * (a[k].r + b[k].r);
    inc[k] += d;
    p[k] += d;
  }
  x[0] = za(x[0], za(zs(a[1], E[0]), zs(b[0], E[1])));
  x[1] = za(x[1], za(zs(a[2], E[0]), zs(b[0], E[2])));
  x[2] = za(x[2], za(zs(a[2], E[1]), zs(b[1], E[2])));
}

template <int TX>
struct Lds {
  static constexpr int TYM = FD_MAXBLOCK / TX;
  static constexpr int W = TX + 2;
  float E[2][3][(TYM + 2) * (TX + 2)];  // E^n, planes k and k+1, over [i0-1, i0+TX] x [j0-1, j0+TY]
  float H[3][(TYM + 1) * (TX + 1)];     // H^{n+1/2} of plane k over [i0-1, i0+TX-1] x [j0-1, j0+TY-1]
  fd_mat mat[FD_MAXMAT];
  double red[FD_MAXBLOCK / 64];
  double ftot[FD_MAXFLUX];  // T(t) partial of the tile per flux plane, stored after the z march
  float probe[FD_MAXPROBE];  // probe samples of the tile, stored after the z march
  // all-axes CPML tiles: x and y grading (1/kappa, b, c at E then H positions) of
  // columns i0-1 .. i0+TX-1 and rows j0-1 .. j0+TYM-1 (0 outside the slabs)
  float gx[6][TX + 1];
  float gy[6][TYM + 1];
};

// ZT: the tile's z range holds z-slab planes.  Without them the z march drops
// every z-CPML test (PMM), so interior tiles of a CPML launch run the same
// code as tiles of a plain launch; the plane below the range still takes the
// general path.
template <int TX, int PM, int GAIN, bool ZT, bool NT>
__device__ void run_tile(const fd_tile& tl, int s_rel, Lds<TX>& s) {
  const cdesc* d = (const cdesc*)tl.d;
  constexpr int W = Lds<TX>::W;
  const int TY = (int)blockDim.x / TX;
  const int t = (int)threadIdx.x;
  const int tx = t % TX, ty = t / TX;
  lds_barrier();  // LDS reuse across tiles of the persistent loop
  // material table: the load is issued here and stored to LDS just before the
  // z march, so its latency overlaps the set-up loads
  const int mwords = d->nmat * (int)(sizeof(fd_mat) / 4);
  const gf* msrc = G((const float*)d->mats);
  const float mword = t < mwords ? msrc[t] : 0.0f;
  const long long n = d->step + s_rel;
  const int par = (int)(n & 1);
  Ctx x;
  make_ctx(x, d, par, PM != 0);
  const int i0 = tl.i0, j0 = tl.j0, k0 = tl.k0, k1 = tl.k1;
  const unsigned gmask = GAIN ? d->gainmask : 0u;
  const size_t ncs = (size_t)d->ncell;
  // field stores: non-temporal (NT) when the launch's working set exceeds the
  // Infinity Cache, so they stream to HBM without displacing lines that are
  // still to be read; a compile-time choice (a runtime branch between the two
  // forms of the same store is merged into the plain one by the compiler)
  auto put = [&](const R32<float>& a, int idx, float v) {
    if constexpr (NT) __builtin_nontemporal_store(v, &a[idx]);
    else a[idx] = v;
  };
  const int i = i0 + tx, j = j0 + ty;
  const bool act = i < x.nx && j < x.ny;
  const int c = j * x.rx + i;
  // the cell's column / row lies on the PEC wall x = 0 / y = 0 (its tangential
  // E components are held at zero there)
  const bool pec_i = !x.px && i == 0, pec_j = !x.py && j == 0;

  // ---- per-tile gather offsets (plane-relative), outside the z loop
  int own_off;
  {
    const int gi = wrap(i, x.nx, x.px), gj = wrap(j, x.ny, x.py);
    own_off = (gi >= 0 && gj >= 0) ? gj * x.rx + gi : -1;
  }
  const int own_slot = (ty + 1) * W + tx + 1;
  // The E staging area has a one-cell ring around the TX x TY tile: ring cell q
  // (bottom row, top row, left column, right column) maps to an LDS slot and a
  // plane offset (-1 beyond a PEC wall).  Thread t stages ring cell t; the
  // launch guarantees 2 (TX + 2) + 2 TY <= blockDim.
  const int nring = 2 * (TX + 2) + 2 * TY;
  auto ring_cell = [&](int q, int& slot, int& off) {
    int lx, ly;
    if (q < TX + 2) { lx = q; ly = 0; }
    else if (q < 2 * (TX + 2)) { lx = q - (TX + 2); ly = TY + 1; }
    else if (q < 2 * (TX + 2) + TY) { lx = 0; ly = 1 + q - 2 * (TX + 2); }
    else { lx = TX + 1; ly = 1 + q - 2 * (TX + 2) - TY; }
    const int gi = wrap(i0 - 1 + lx, x.nx, x.px), gj = wrap(j0 - 1 + ly, x.ny, x.py);
    slot = ly * W + lx;
    off = (gi >= 0 && gj >= 0) ? gj * x.rx + gi : -1;
  };
  int r_slot = -1, r_off = -1;
  if (t < nring) ring_cell(t, r_slot, r_off);
  // halo duty: threads [0, TX) own the row j0-1, threads [TX, TX+TY) the column
  // i0-1; hr: column of the row cell / row of the column cell
  const bool bh = t < TX;
  const bool lh = !bh && t < TX + TY;
  const int hr = lh ? t - TX : t;
  const int hgi = wrap(lh ? i0 - 1 : i0 + hr, x.nx, x.px);
  const int hgj = wrap(lh ? j0 + hr : j0 - 1, x.ny, x.py);
  const bool hact = (lh || bh) && hgi >= 0 && hgj >= 0 && (lh ? (j0 + hr < x.ny) : (i0 + hr < x.nx));
  const int h_off = hact ? hgj * x.rx + hgi : 0;

  // ---- sources, probes and flux planes that touch the tile (set on the host);
  // srcmine: the sources that drive this thread's column
  const unsigned srcmask = tl.srcmask, pmask = tl.pmask, fmask = tl.fmask;
  unsigned srcmine = 0u;
  for (unsigned mm = srcmask; mm; mm &= mm - 1u) {
    const int q = __builtin_ctz(mm);
    if (d->src_kind[q] != 0 || d->src_cell[q] == c) srcmine |= 1u << q;  // sheets drive every column
  }
  const bool edue = d->ke > 0 && (n % d->ke) == 0;
  double eacc = 0.0;

  // ---- staging.  Iteration k of the z march consumes a Stage holding E^n of
  // plane k+1 (own cell and one ring cell; stored to LDS at the top of the
  // iteration) and the own inputs of plane k (H^{n-1/2}, the halo-duty H, the
  // material index).  Two Stages alternate, so the loads for plane k+3 (E) and
  // k+2 (own inputs) are in flight while plane k is computed: the global-load
  // latency is spread over two iterations.  Slots outside the grid hold the
  // periodic image or 0.
  // A Stage holds raw load results; validity selects are applied where the
  // values are used, so no instruction touches a load result before it is due.
  struct Stage {
    float own[3];
    float ring[3];
    bool zok;     // plane inside the grid (or its periodic image)
    float ho[3];  // H^{n-1/2} of the own cell
    float hsel;   // halo-duty cell: Hy (column cell) or Hx (row cell)
    float hh2;    // halo-duty cell: Hz
    int m;
    float ph[2];  // z-slab planes: old psi_H of Hx, Hy (own)
    float phz;    // z-slab planes: old psi_H of hsel's z difference at the halo-duty cell
    float pe[2];  // z-slab planes: old psi_E of Ex, Ey (own)
    float gh[3];  // z-slab planes: H-side grading 1/kappa, b, c (uniform)
    float ge[3];  // z-slab planes: E-side grading (uniform)
    uint32_t gi;  // gain cells: the cell's gain ordinal (index of its gain state)
  };
  // Every global load of the z march is issued whatever the lane's own cell (a
  // lane with nothing to load reads element 0 and discards it; only uniform
  // conditions -- the all-axes tile's slabs -- skip loads), and the march stores to
  // global memory only the fields and CPML memory: the loads in flight per
  // iteration are then the same on every path, so the compiler waits for
  // exactly the Stage it consumes and leaves the other one in flight.
  // live = false: the plane is past the tile; the loads are still issued (at
  // element 0) so that every path through the march issues the same loads.
  // Linear tiles without x / y CPML (EREG) keep the own cell's E^n of planes k
  // and k+1 in registers and form each load address with one select: in-plane
  // offsets are clamped to cell 0 once where the lane has nothing to load (its
  // values are discarded at use).  The other classes, near their register caps,
  // read those E values from LDS and select per load.  Either way a plane the
  // march does not need (past the tile, or outside the CPML slabs for psi) is
  // read at element 0 by every lane: one cache line, not a row of another plane.
  constexpr bool EREG = GAIN == 0 && !(ZT && PM == 7);
  const uint32_t own_l = own_off >= 0 ? own_off : 0, ring_l = r_off >= 0 ? r_off : 0;
  const uint32_t c_l = act ? c : 0;  // h_off is already 0 without halo duty
  auto load_e = [&](int kk, Stage& S, bool live) {
    const int kz = kk < x.nz ? kk : (x.pz ? kk - x.nz : -1);
    S.zok = kz >= 0;
    const uint32_t zo = S.zok ? kz * x.plane : 0;
    const uint32_t io = EREG ? (live ? zo + own_l : 0u) : ((live && own_off >= 0) ? zo + own_off : 0u);
    const uint32_t ir = EREG ? (live ? zo + ring_l : 0u) : ((live && r_off >= 0) ? zo + r_off : 0u);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) S.own[cc] = x.Ein[cc][io];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) S.ring[cc] = x.Ein[cc][ir];
  };
  // stages E^n of the Stage's plane into LDS buffer b; eown receives the own
  // cell's values (0 beyond a PEC wall), which the march keeps in registers
  auto store_e = [&](int b, const Stage& S, float eown[3]) {
    const bool oko = S.zok && own_off >= 0, okr = S.zok && r_off >= 0;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      eown[cc] = oko ? S.own[cc] : 0.0f;
      s.E[b][cc][own_slot] = eown[cc];
    }
    if (r_slot >= 0) {
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) s.E[b][cc][r_slot] = okr ? S.ring[cc] : 0.0f;
    }
  };
  const R32<const uint8_t> matp{(const gu8*)d->mat};
  const R32<const uint32_t> gidxp{(const __attribute__((address_space(1))) uint32_t*)d->gidx};
  constexpr int PMM = ZT ? PM : (PM & 3);  // CPML axes the march handles
  constexpr bool ZP = ZT && PM == 4;       // z-slab psi prefetched with the plane (z-only CPML tiles)
  constexpr bool AX = PMM == 7;            // all-axes CPML tiles: psi of the plane issued up front
  static_assert(PMM == 0 || PMM == 4 || PMM == 7, "tile classes: no CPML, z slabs, all axes");
  auto load_h = [&](int kk, Stage& S, bool live) {
    kk = live ? kk : 0;
    const uint32_t zo = kk * x.plane;
    const uint32_t io = EREG ? (live ? zo + c_l : 0u) : ((live && act) ? zo + c : 0u);
    const uint32_t ih = EREG ? (live ? zo + h_off : 0u) : ((live && hact) ? zo + h_off : 0u);
#pragma unroll
    for (int q = 0; q < 3; ++q) S.ho[q] = x.Hin[q][io];
    S.m = matp[io];  // lanes outside the grid read cell 0: a valid material
    if (GAIN) S.gi = gidxp[io];
    // the column i0-1 needs Hy, Hz; the row j0-1 needs Hx, Hz.  The lane picks
    // the array (a choice between two loaded values would wait for both loads
    // at once, and a choice between two Stage fields becomes an indexed, spilled
    // access)
    S.hsel = R32<const float>{lh ? x.Hin[1].p : x.Hin[0].p}[ih];
    S.hh2 = x.Hin[2][ih];
    if (ZP) {
      // the z differences of Hx, Hy, Ex, Ey in a z slab carry psi: load the
      // old values with the plane's other inputs (psi_E is touched only by the
      // owner of the cell, so reading it early is safe); the grading is uniform
      const int sz = slab(x, 2, kk);
      const int nz = x.n[2];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        S.ge[q] = x.prof[2][q * nz + kk];
        S.gh[q] = x.prof[2][(3 + q) * nz + kk];
      }
      const bool in = live && sz >= 0;
      const uint32_t base = in ? sz * x.plane : 0;
      const uint32_t jo = EREG ? (in ? base + c_l : 0u) : ((in && act) ? base + c : 0u);
      const uint32_t jh = EREG ? (in ? base + h_off : 0u) : ((in && hact) ? base + h_off : 0u);
      S.ph[0] = x.psiHin[2][fam(0, 2)][jo];
      S.ph[1] = x.psiHin[2][fam(1, 2)][jo];
      S.pe[0] = x.psiE[2][fam(0, 2)][jo];
      S.pe[1] = x.psiE[2][fam(1, 2)][jo];
      S.phz = R32<const float>{lh ? x.psiHin[2][fam(1, 2)].p : x.psiHin[2][fam(0, 2)].p}[jh];
    }
  };

  // Loads are issued in the order their values are consumed (the memory
  // counter retires in order): plane k0, the inputs of H^{n+1/2} at plane
  // k0-1 (the march carries H of the plane below), then the two Stages.
  Stage SA, SB;
  load_e(k0, SA, true);
  const int km = prv(k0, x.nz, x.pz);
  const bool pro = act && km >= 0;
  const int jp = nxt(j, x.ny, x.py), ip = nxt(i, x.nx, x.px);
  float pEz, pEzj, pEzi, pEy, pEx, pHx, pHy;
  {
    const int zm = pro ? km * x.plane : 0;
    const uint32_t om = pro ? zm + c : 0;
    const uint32_t ojp = (pro && jp >= 0) ? zm + jp * x.rx + i : 0;
    const uint32_t oip = (pro && ip >= 0) ? zm + j * x.rx + ip : 0;
    pEz = x.Ein[2][om];
    pEzj = x.Ein[2][ojp];
    pEzi = x.Ein[2][oip];
    pEy = x.Ein[1][om];
    pEx = x.Ein[0][om];
    pHx = x.Hin[0][om];
    pHy = x.Hin[1][om];
  }
  // all-axes tiles: the CPML inputs of H at plane k0-1 and this thread's first
  // entry of the x / y grading tables, issued now so that their latency
  // overlaps the loads above instead of following them
  PreStretch px1{}, px2{}, py1{}, py2{};
  float gxv = 0.0f, gyv = 0.0f;
  if (AX) {
    px1 = pre_load<PM>(x, 0, 1, j, i, j, km, pro);
    px2 = pre_load<PM>(x, 0, 2, km, i, j, km, pro);
    py1 = pre_load<PM>(x, 1, 2, km, i, j, km, pro);
    py2 = pre_load<PM>(x, 1, 0, i, i, j, km, pro);
    if (x.t[0] > 0) {
      const int r = t / (TX + 1), ii = i0 - 1 + t % (TX + 1);
      const bool ok = t < 6 * (TX + 1) && ii >= 0 && ii < x.nx && slab(x, 0, ii) >= 0;
      const float v = x.prof[0][ok ? r * x.nx + ii : 0];
      gxv = ok ? v : 0.0f;
    }
    if (x.t[1] > 0) {
      constexpr int GY = Lds<TX>::TYM + 1;
      const int r = t / GY, jj = j0 - 1 + t % GY;
      const bool ok = t < 6 * GY && jj >= 0 && jj < x.ny && slab(x, 1, jj) >= 0;
      const float v = x.prof[1][ok ? r * x.ny + jj : 0];
      gyv = ok ? v : 0.0f;
    }
  }
  float ecur[3];  // E^n of the own cell at the plane being marched
  store_e(0, SA, ecur);
  load_e(k0 + 1, SA, true);
  load_h(k0, SA, true);
  load_e(k0 + 2, SB, k0 + 1 < k1);
  load_h(k0 + 1, SB, k0 + 1 < k1);
  // H^{n+1/2} at (i, j, k0-1); E^n at (i, j, k0) is already in LDS buffer 0
  float hxm = 0.0f, hym = 0.0f;
  if (AX) {
    const float ey1 = ecur[1], ex1 = ecur[0];
    const float ezj = jp >= 0 ? pEzj : 0.0f, ezi = ip >= 0 ? pEzi : 0.0f;
    const float hx = fmaf(-x.ch, pre_apply(px1, ezj - pEz) - pre_apply(px2, ey1 - pEy), pHx);
    const float hy = fmaf(-x.ch, pre_apply(py1, ex1 - pEx) - pre_apply(py2, ezi - pEz), pHy);
    hxm = pro ? hx : 0.0f;
    hym = pro ? hy : 0.0f;
  } else if (pro) {
    const float ey1 = ecur[1], ex1 = ecur[0];
    const float ezj = jp >= 0 ? pEzj : 0.0f, ezi = ip >= 0 ? pEzi : 0.0f;
    hxm = h_from<PM>(x, 0, 1, j, 2, km, i, j, km, ezj, pEz, ey1, pEy, pHx, false);
    hym = h_from<PM>(x, 1, 2, km, 0, i, i, j, km, ex1, pEx, ezi, pEz, pHy, false);
  }

  // plane k uses LDS E buffer cb = (k - k0) & 1, a compile-time constant in
  // each of the two unrolled copies, so every LDS address is a fixed offset
  {
    float* mdst = reinterpret_cast<float*>(s.mat);
    if (t < mwords) mdst[t] = mword;
    for (int q = t + (int)blockDim.x; q < mwords; q += (int)blockDim.x) mdst[q] = msrc[q];
  }
  // all-axes CPML: slab indices of the own column and of the halo-duty cell along
  // x and y (fixed over the march), and the tile's x / y grading tables in LDS
  int sxo = -1, syo = -1, sxh = -1, syh = -1;
  // uniform: the tile's columns (with the halo column i0-1) reach an x slab,
  // its rows (with the halo row j0-1) a y slab
  const bool uxs = AX && x.t[0] > 0 && (i0 - 1 < x.lo[0] || i0 + TX > x.nx - x.hi[0]);
  const bool uys = AX && x.t[1] > 0 && (j0 - 1 < x.lo[1] || j0 + TY > x.ny - x.hi[1]);
  if (AX) {
    sxo = slab(x, 0, i);
    syo = slab(x, 1, j);
    if (hact) {
      sxh = slab(x, 0, hgi);
      syh = slab(x, 1, hgj);
    }
    if (t < 6 * (TX + 1)) s.gx[t / (TX + 1)][t % (TX + 1)] = gxv;
    for (int q = t + (int)blockDim.x; q < 6 * (TX + 1); q += (int)blockDim.x) {
      const int r = q / (TX + 1), ii = i0 - 1 + q % (TX + 1);
      s.gx[r][q % (TX + 1)] = (ii >= 0 && ii < x.nx && slab(x, 0, ii) >= 0) ? x.prof[0][r * x.nx + ii] : 0.0f;
    }
    if (t < 6 * (Lds<TX>::TYM + 1)) s.gy[t / (Lds<TX>::TYM + 1)][t % (Lds<TX>::TYM + 1)] = gyv;
    for (int q = t + (int)blockDim.x; q < 6 * (Lds<TX>::TYM + 1); q += (int)blockDim.x) {
      const int r = q / (Lds<TX>::TYM + 1), jj = j0 - 1 + q % (Lds<TX>::TYM + 1);
      s.gy[r][q % (Lds<TX>::TYM + 1)] = (jj >= 0 && jj < x.ny && slab(x, 1, jj) >= 0) ? x.prof[1][r * x.ny + jj] : 0.0f;
    }
  }

  auto plane_step = [&](auto cbc, const int k, Stage& S) __attribute__((always_inline)) {
    constexpr int cb = decltype(cbc)::value;
    constexpr int nb = cb ^ 1;
    // plane k+1 into LDS; the loads two planes ahead reuse the same Stage
    float enx[3];  // E^n of the own cell at plane k+1
    store_e(nb, S, enx);
    const int zo = k * x.plane;
    const int o = zo + c;
    const int sz = (ZP || AX) ? slab(x, 2, k) : -1;
    // all-axes CPML: the old psi the plane needs, issued before the barriers
    // (lanes outside a slab read element 0); z grading is uniform over the plane
    float aH[6] = {}, aE[6] = {}, aHh[4] = {}, gzE[3] = {}, gzH[3] = {};
    uint32_t ox = 0, oy = 0, oz = 0, ohx = 0, ohy = 0, ohz = 0;
    if (AX) {
      ox = (act && sxo >= 0) ? (uint32_t)((k * x.ny + j) * x.t[0] + sxo) : 0u;
      oy = (act && syo >= 0) ? (uint32_t)((k * x.t[1] + syo) * x.nx + i) : 0u;
      oz = (act && sz >= 0) ? (uint32_t)(sz * x.plane + c) : 0u;
      ohx = (hact && sxh >= 0) ? (uint32_t)((k * x.ny + hgj) * x.t[0] + sxh) : 0u;
      ohy = (hact && syh >= 0) ? (uint32_t)((k * x.t[1] + syh) * x.nx + hgi) : 0u;
      ohz = (hact && sz >= 0) ? (uint32_t)(sz * x.plane + h_off) : 0u;
      // own H: Hx(y, z), Hy(z, x), Hz(x, y); own E in the same order.  The
      // reads of an axis whose slabs neither the tile (x, y) nor the plane (z)
      // touches are skipped (uniform branches; the values stay 0 and unused)
      // halo: column cells (lh) need Hy(z, x), row cells Hx(y, z); both need Hz(x, y)
      if (uxs) {
        aH[3] = x.psiHin[0][0][ox];
        aH[4] = x.psiHin[0][1][ox];
        aE[3] = x.psiE[0][0][ox];
        aE[4] = x.psiE[0][1][ox];
        aHh[2] = x.psiHin[0][1][ohx];
      }
      if (uys) {
        aH[0] = x.psiHin[1][1][oy];
        aH[5] = x.psiHin[1][0][oy];
        aE[0] = x.psiE[1][1][oy];
        aE[5] = x.psiE[1][0][oy];
        aHh[3] = x.psiHin[1][0][ohy];
      }
      if (uxs | uys) {
        const gf* pc1o = lh ? x.psiHin[0][0].p : x.psiHin[1][1].p;
        aHh[1] = pc1o[lh ? ohx : ohy];
      }
      if (sz >= 0) {
        aH[1] = x.psiHin[2][0][oz];
        aH[2] = x.psiHin[2][1][oz];
        aE[1] = x.psiE[2][0][oz];
        aE[2] = x.psiE[2][1][oz];
        const gf* pc1z = lh ? x.psiHin[2][1].p : x.psiHin[2][0].p;
        aHh[0] = pc1z[ohz];
      }
      if (sz >= 0) {  // uniform: the z grading exists only with z slabs
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          gzE[q] = x.prof[2][q * x.nz + k];
          gzH[q] = x.prof[2][(3 + q) * x.nz + k];
        }
      }
    }
    // gain-cell inputs of plane k (populations, P^n, P^{n-1}), consumed in the E
    // update; other lanes read element 0
    float gnh[3], gnl[3], gPn[3], gPm[3];
    bool gk = false;
    if (GAIN) {
      gk = act && ((gmask >> S.m) & 1u);
      const uint32_t ig = gk ? S.gi : 0u;
      const gf* pop = G(d->pop);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        gnh[q] = pop[(size_t)q * ncs + ig];
        gnl[q] = pop[(size_t)(3 + q) * ncs + ig];
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        gPn[q] = G((const float*)d->P[par][q])[ig];
        gPm[q] = G((const float*)d->P[par ^ 1][q])[ig];
      }
    }
    // the loads two planes ahead go out after this plane's psi and gain inputs:
    // the memory counter retires in order, so waiting for those does not wait
    // for them
    load_e(k + 3, S, k + 2 < k1);
    // E^n of the own cell at plane k, from registers or read from LDS before the
    // second barrier (after it a faster wave may already be staging plane k+2
    // into this buffer)
    float eo[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) eo[q] = EREG ? ecur[q] : s.E[cb][q][own_slot];
    lds_barrier();
    // ---- H^{n+1/2} of plane k: own cell and halo duty
    float hx = 0.0f, hy = 0.0f, hz = 0.0f;
    {
      const float* Ex = s.E[cb][0];
      const float* Ey = s.E[cb][1];
      const float* Ez = s.E[cb][2];
      const float* Ex1 = s.E[nb][0];
      const float* Ey1 = s.E[nb][1];
      const int a = own_slot;
      // own-cell E^n at planes k and k+1: registers in the classes that carry
      // them, else the LDS copies (equal values; the capped classes are short
      // of registers)
      const float e0x = EREG ? eo[0] : Ex[a], e0y = EREG ? eo[1] : Ey[a], e0z = EREG ? eo[2] : Ez[a];
      const float e1x = EREG ? enx[0] : Ex1[a], e1y = EREG ? enx[1] : Ey1[a];
      if (act && AX) {
        const int xi = tx + 1, yj = ty + 1;
        const float* gxh[3] = {s.gx[3], s.gx[4], s.gx[5]};
        const float* gyh[3] = {s.gy[3], s.gy[4], s.gy[5]};
        float d1 = Ez[a + W] - e0z, d2 = e1y - e0y;
        d1 = stretch_v(d1, syo, gyh[0][yj], gyh[1][yj], gyh[2][yj], aH[0], true, x.psiHout[1][1], oy);
        d2 = stretch_v(d2, sz, gzH[0], gzH[1], gzH[2], aH[1], true, x.psiHout[2][0], oz);
        hx = fmaf(-x.ch, d1 - d2, S.ho[0]);
        d1 = e1x - e0x;
        d2 = Ez[a + 1] - e0z;
        d1 = stretch_v(d1, sz, gzH[0], gzH[1], gzH[2], aH[2], true, x.psiHout[2][1], oz);
        d2 = stretch_v(d2, sxo, gxh[0][xi], gxh[1][xi], gxh[2][xi], aH[3], true, x.psiHout[0][0], ox);
        hy = fmaf(-x.ch, d1 - d2, S.ho[1]);
        d1 = Ey[a + 1] - e0y;
        d2 = Ex[a + W] - e0x;
        d1 = stretch_v(d1, sxo, gxh[0][xi], gxh[1][xi], gxh[2][xi], aH[4], true, x.psiHout[0][1], ox);
        d2 = stretch_v(d2, syo, gyh[0][yj], gyh[1][yj], gyh[2][yj], aH[5], true, x.psiHout[1][0], oy);
        hz = fmaf(-x.ch, d1 - d2, S.ho[2]);
        put(x.Hout[0], o, hx);
        put(x.Hout[1], o, hy);
        put(x.Hout[2], o, hz);
      } else if (PMM == 0) {
        // no CPML memory: every lane computes (lanes outside the grid read
        // in-bounds LDS slots and element 0 of H) and only the stores are masked
        hx = h_from<0>(x, 0, 1, j, 2, k, i, j, k, Ez[a + W], e0z, e1y, e0y, S.ho[0], true);
        hy = h_from<0>(x, 1, 2, k, 0, i, i, j, k, e1x, e0x, Ez[a + 1], e0z, S.ho[1], true);
        hz = h_from<0>(x, 2, 0, i, 1, j, i, j, k, Ey[a + 1], e0y, Ex[a + W], e0x, S.ho[2], true);
        hx = act ? hx : 0.0f;
        hy = act ? hy : 0.0f;
        hz = act ? hz : 0.0f;
        if (act) {
          put(x.Hout[0], o, hx);
          put(x.Hout[1], o, hy);
          put(x.Hout[2], o, hz);
        }
      } else if (act) {
        hx = h_from<PMM, ZP>(x, 0, 1, j, 2, k, i, j, k, Ez[a + W], e0z, e1y, e0y, S.ho[0], true, sz, c, S.ph[0], S.gh);
        hy = h_from<PMM, ZP>(x, 1, 2, k, 0, i, i, j, k, e1x, e0x, Ez[a + 1], e0z, S.ho[1], true, sz, c, S.ph[1], S.gh);
        hz = h_from<PMM, ZP>(x, 2, 0, i, 1, j, i, j, k, Ey[a + 1], e0y, Ex[a + W], e0x, S.ho[2], true, sz, c, 0.0f, S.gh);
        put(x.Hout[0], o, hx);
        put(x.Hout[1], o, hy);
        put(x.Hout[2], o, hz);
      }
      const int hs = (ty + 1) * (TX + 1) + tx + 1;
      s.H[0][hs] = hx;
      s.H[1][hs] = hy;
      s.H[2][hs] = hz;
      if (hact && AX) {
        // column cell (i0-1, j0+hr): Hy(z, x) and Hz(x, y); row cell (i0+hr, j0-1):
        // Hx(y, z) and Hz(x, y).  One path, operands selected per lane (the
        // column's x-table entry is 0 and its y-table entry hr+1, the row's the
        // reverse); bit-identical to separate column and row paths
        const int b = lh ? (hr + 1) * W : hr + 1;  // E slot of the halo cell
        const int xe = lh ? 0 : hr + 1, ye = lh ? hr + 1 : 0;
        const float* z1 = lh ? Ex1 : Ey1;
        const float* z0 = lh ? Ex : Ey;
        float zd = z1[b] - z0[b];
        zd = stretch_v(zd, sz, gzH[0], gzH[1], gzH[2], aHh[0], false, x.psiHout[2][0], 0u);
        // the transverse difference of Ez: along x for the column, along y for the row
        float td = Ez[b + (lh ? 1 : W)] - Ez[b];
        td = stretch_v(td, lh ? sxh : syh, lh ? s.gx[3][0] : s.gy[3][0], lh ? s.gx[4][0] : s.gy[4][0],
                       lh ? s.gx[5][0] : s.gy[5][0], aHh[1], false, x.psiHout[0][0], 0u);
        const float v1 = fmaf(-x.ch, lh ? zd - td : td - zd, S.hsel);
        float d1 = Ey[b + 1] - Ey[b];
        float d2 = Ex[b + W] - Ex[b];
        d1 = stretch_v(d1, sxh, s.gx[3][xe], s.gx[4][xe], s.gx[5][xe], aHh[2], false, x.psiHout[0][1], 0u);
        d2 = stretch_v(d2, syh, s.gy[3][ye], s.gy[4][ye], s.gy[5][ye], aHh[3], false, x.psiHout[1][0], 0u);
        const float hzv = fmaf(-x.ch, d1 - d2, S.hh2);
        const int hb = lh ? (hr + 1) * (TX + 1) : hr + 1;  // H slot of the halo cell
        (lh ? s.H[1] : s.H[0])[hb] = v1;
        s.H[2][hb] = hzv;
      } else if (hact) {
        // the column cell (i0-1, j0+hr) takes Hy and Hz, the row cell (i0+hr, j0-1)
        // Hx and Hz: one path for both, operands selected per lane.  The first
        // component is -(dt/dx)(z difference - transverse difference of Ez) for
        // the column and -(dt/dx)(y difference of Ez - z difference) for the row;
        // bit-identical to the two h_from calls it replaces
        const int b = lh ? (hr + 1) * W : hr + 1;  // E slot of the halo cell
        const float* z1 = lh ? Ex1 : Ey1;
        const float* z0 = lh ? Ex : Ey;
        float zd = z1[b] - z0[b];
        if (ZP) zd = stretch_z<true>(x, 0, S.gh, sz, h_off, zd, false, S.phz);
        const float td = Ez[b + (lh ? 1 : W)] - Ez[b];
        const float v1 = fmaf(-x.ch, lh ? zd - td : td - zd, S.hsel);
        const float hzv = fmaf(-x.ch, (Ey[b + 1] - Ey[b]) - (Ex[b + W] - Ex[b]), S.hh2);
        const int hb = lh ? (hr + 1) * (TX + 1) : hr + 1;  // H slot of the halo cell
        (lh ? s.H[1] : s.H[0])[hb] = v1;
        s.H[2][hb] = hzv;
      }
    }
    lds_barrier();
    // ---- E^{n+1} of plane k (own cell)
    float ex_n = 0.0f, ey_n = 0.0f, ez_n = 0.0f;
    if (act) {
      const int hs = (ty + 1) * (TX + 1) + tx + 1;
      const float hz_im = s.H[2][hs - 1], hy_im = s.H[1][hs - 1];
      const float hx_jm = s.H[0][hs - (TX + 1)], hz_jm = s.H[2][hs - (TX + 1)];
      const fd_mat& mt = s.mat[S.m];
      float dP[3] = {0.0f, 0.0f, 0.0f};
      float Pnew[3] = {0.0f, 0.0f, 0.0f};
      const bool g = GAIN && gk;
      float nh[3] = {0.0f, 0.0f, 0.0f}, nl[3] = {0.0f, 0.0f, 0.0f};
      if (g) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          nh[q] = gnh[q];
          nl[q] = gnl[q];
        }
      }
      if (GAIN == 1 && g) {
        const float n1 = nh[0] + nl[0], n2 = nh[1] + nl[1];
        float F[3] = {0.0f, 0.0f, 0.0f};
        if (mt.noise != 0.0f) {
          float gg[3];
          // the counter takes the dense cell index (k ny + j) nx + i
          normals3((uint32_t)n, ((uint32_t)k * (uint32_t)x.ny + (uint32_t)j) * (uint32_t)x.nx + (uint32_t)i,
                   d->key0, d->key1, gg);
          const float amp = mt.noise * sqrtf(fmaxf(n2, 0.0f));
#pragma unroll
          for (int q = 0; q < 3; ++q) F[q] = amp * gg[q];
        }
        const float dn = n1 - n2;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const float Pn = gPn[q];
          const float Pm = gPm[q];
          Pnew[q] = fmaf(mt.C1, Pn, fmaf(mt.C2, Pm, fmaf(mt.C3k * dn, eo[q], mt.C3 * F[q])));
          dP[q] = Pnew[q] - Pn;
        }
      }
      float cx = 0.0f, cy = 0.0f, cz = 0.0f;  // source terms dx*J of this cell
      for (unsigned mm = srcmask; mm; mm &= mm - 1u) {  // uniform; scalar loads only
        const int q = __builtin_ctz(mm);
        if (d->src_k[q] != k) continue;
        float v = n < d->src_len[q] ? ((const cfloat*)d->src_tab[q])[n] : 0.0f;
        if (!((srcmine >> q) & 1u)) continue;
        if (d->src_kind[q] == 2) v *= G(d->src_prof[q])[c];  // beam: transverse waist profile
        const int sc = d->src_comp[q];
        if (sc == 0) cx += v;
        else if (sc == 1) cy += v;
        else cz += v;
      }
      // av: E^{n+1} without the polarization current; on: not a PEC-held component
      float av[3] = {0.0f, 0.0f, 0.0f};
      bool on[3] = {false, false, false};
      if (PMM == 0) {
        // no CPML memory: plain selects for the components held by a PEC wall
        const bool pec_k = !x.pz && k == 0;  // uniform over the plane
        on[0] = !(pec_j | pec_k);
        on[1] = !(pec_k | pec_i);
        on[2] = !(pec_i | pec_j);
        const float v0 = fmaf(mt.cb, ((hz - hz_jm) - (hy - hym)) - cx, eo[0]);
        const float v1 = fmaf(mt.cb, ((hx - hxm) - (hz - hz_im)) - cy, eo[1]);
        const float v2 = fmaf(mt.cb, ((hy - hy_im) - (hx - hx_jm)) - cz, eo[2]);
        av[0] = on[0] ? v0 : 0.0f;
        av[1] = on[1] ? v1 : 0.0f;
        av[2] = on[2] ? v2 : 0.0f;
      } else {
      if (!(pec_j || (!x.pz && k == 0))) {  // Ex: d/dy Hz - d/dz Hy
        float d1 = hz - hz_jm, d2 = hy - hym;
        if (AX) {
          d1 = stretch_v(d1, syo, s.gy[0][ty + 1], s.gy[1][ty + 1], s.gy[2][ty + 1], aE[0], true, x.psiE[1][1], oy);
          d2 = stretch_v(d2, sz, gzE[0], gzE[1], gzE[2], aE[1], true, x.psiE[2][0], oz);
        } else if (PMM) {
          d1 = stretch<false, PMM>(x, 0, 1, j, i, j, k, d1, true);
          d2 = ZP ? stretch_z<false>(x, 0, S.ge, sz, c, d2, true, S.pe[0]) : stretch<false, PMM>(x, 0, 2, k, i, j, k, d2, true);
        }
        av[0] = fmaf(mt.cb, (d1 - d2) - cx, eo[0]);
        on[0] = true;
      }
      if (!((!x.pz && k == 0) || pec_i)) {  // Ey: d/dz Hx - d/dx Hz
        float d1 = hx - hxm, d2 = hz - hz_im;
        if (AX) {
          d1 = stretch_v(d1, sz, gzE[0], gzE[1], gzE[2], aE[2], true, x.psiE[2][1], oz);
          d2 = stretch_v(d2, sxo, s.gx[0][tx + 1], s.gx[1][tx + 1], s.gx[2][tx + 1], aE[3], true, x.psiE[0][0], ox);
        } else if (PMM) {
          d1 = ZP ? stretch_z<false>(x, 1, S.ge, sz, c, d1, true, S.pe[1]) : stretch<false, PMM>(x, 1, 2, k, i, j, k, d1, true);
          d2 = stretch<false, PMM>(x, 1, 0, i, i, j, k, d2, true);
        }
        av[1] = fmaf(mt.cb, (d1 - d2) - cy, eo[1]);
        on[1] = true;
      }
      if (!(pec_i || pec_j)) {  // Ez: d/dx Hy - d/dy Hx
        float d1 = hy - hy_im, d2 = hx - hx_jm;
        if (AX) {
          d1 = stretch_v(d1, sxo, s.gx[0][tx + 1], s.gx[1][tx + 1], s.gx[2][tx + 1], aE[4], true, x.psiE[0][1], ox);
          d2 = stretch_v(d2, syo, s.gy[0][ty + 1], s.gy[1][ty + 1], s.gy[2][ty + 1], aE[5], true, x.psiE[1][0], oy);
        } else if (PMM) {
          d1 = stretch<false, PMM>(x, 2, 0, i, i, j, k, d1, true);
          d2 = stretch<false, PMM>(x, 2, 1, j, i, j, k, d2, true);
        }
        av[2] = fmaf(mt.cb, (d1 - d2) - cz, eo[2]);
        on[2] = true;
      }
      }
      if (GAIN == 0) {
        // no polarization current: av is E^{n+1} (0 where a PEC wall holds it),
        // bit for bit what av - 0 / eps gives
        ex_n = av[0];
        ey_n = av[1];
        ez_n = av[2];
      } else {
        if (on[0]) ex_n = av[0] - dP[0] * mt.inv_eps;
        if (on[1]) ey_n = av[1] - dP[1] * mt.inv_eps;
        if (on[2]) ez_n = av[2] - dP[2] * mt.inv_eps;
      }
      put(x.Eout[0], o, ex_n);
      put(x.Eout[1], o, ey_n);
      put(x.Eout[2], o, ez_n);
      if (GAIN == 1 && g) {
        const float en[3] = {ex_n, ey_n, ez_n};
        float u = 0.0f;
#pragma unroll
        for (int q = 0; q < 3; ++q) u = fmaf(0.5f * (eo[q] + en[q]), dP[q] * mt.inv_dt, u);
        const float nn[4] = {1.0f - ((nh[0] + nh[1]) + nh[2]) - ((nl[0] + nl[1]) + nl[2]),
                             nh[0] + nl[0], nh[1] + nl[1], nh[2] + nl[2]};
        const int nc = d->ncell;
        gf* pop = G(d->pop);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          float inc = mt.Bu[r] * u;
#pragma unroll
          for (int q = 0; q < 4; ++q) inc = fmaf(mt.MI[r][q], nn[q], inc);
          two_sum(nh[r], nl[r], inc);
          pop[(size_t)r * nc + S.gi] = nh[r];
          pop[(size_t)(3 + r) * nc + S.gi] = nl[r];
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) G(d->P[par ^ 1][q])[S.gi] = Pnew[q];
      }
      for (unsigned mm = pmask; mm; mm &= mm - 1u) {  // uniform
        const int p = __builtin_ctz(mm);
        if (d->probe_k[p] != k || d->probe_cell[p] != c) continue;
        const int cp = d->probe_comp[p];
        s.probe[p] = cp == 0 ? ex_n : cp == 1 ? ey_n : cp == 2 ? ez_n : cp == 3 ? hx : cp == 4 ? hy : hz;
      }
      if (edue) {
        const float e2 = fmaf(eo[0], eo[0], fmaf(eo[1], eo[1], eo[2] * eo[2]));
        const float hh = fmaf(S.ho[0], hx, fmaf(S.ho[1], hy, S.ho[2] * hz));
        eacc += (double)(mt.eps * e2) + (double)hh;
      }
    }
    // own inputs two planes ahead into the Stage just consumed
    load_h(k + 2, S, k + 2 < k1);
    // transmitted power through flux planes at this k (uniform branch)
    if (fmask) {
      for (int f = 0; f < FD_MAXFLUX; ++f) {
        if (!((fmask >> f) & 1u) || d->flux_k[f] != k) continue;
        double v = 0.0;
        if (act) {
          const float sx = 0.5f * (eo[0] + ex_n), sy = 0.5f * (eo[1] + ey_n);
          const float hyc = 0.5f * (hym + hy), hxc = 0.5f * (hxm + hx);
          v = (double)(sx * hyc) - (double)(sy * hxc);
        }
        const double tot = block_sum(v, s.red);
        if (t == 0) s.ftot[f] = tot;
      }
    }
    hxm = hx;
#pragma unroll
    for (int q = 0; q < 3; ++q) ecur[q] = enx[q];
    hym = hy;
  };

  // the loop body is both copies unconditionally (a path that skips the second
  // copy would make the compiler wait for every load at the loop head)
  int k = k0;
  for (; k + 1 < k1; k += 2) {
    plane_step(std::integral_constant<int, 0>(), k, SA);
    plane_step(std::integral_constant<int, 1>(), k + 1, SB);
  }
  if (k < k1) plane_step(std::integral_constant<int, 0>(), k, SA);
  // probe samples and T(t) partials gathered during the march
  if (pmask | fmask) {
    lds_barrier();
    if (t < FD_MAXPROBE && ((pmask >> t) & 1u)) G(d->probe_ring)[(long long)t * d->max_steps + n] = s.probe[t];
    if (t < FD_MAXFLUX && ((fmask >> t) & 1u)) G(d->flux_T[t])[n * d->nblk + tl.blk] = s.ftot[t];
  }
  if (edue) {
    const double tot = block_sum(eacc, s.red);
    if (t == 0) G(d->energy)[(n / d->ke) * d->ntiles + tl.tidx] = tot;
  }
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup w runs on XCD
// w mod 8), and each XCD has its own L2.  Renumber so that XCD x walks one
// contiguous eighth of the tile list: tiles adjacent in the list (x, y and z
// neighbours, whose halos overlap) then share an L2.  A bijection on [0, n).
__device__ __forceinline__ int xcd_tile(int w, int n) {
  constexpr int kXcd = 8;
  const int q = n / kXcd, r = n % kXcd;
  const int x = w % kXcd, s = w / kXcd;
  return x * q + (x < r ? x : r) + s;
}

// With a cost-balanced partition (use_part), workgroup w takes tile
// part.start[x] + w/8 of XCD x = w mod 8, or nothing if that part is shorter;
// otherwise the workgroups loop over the renumbered tile list.
template <int TX, int PM, int GAIN, bool NT>
__device__ __forceinline__ void step_body(const fd_tile* __restrict__ tiles, int ntiles, int s, const fd_xcd& part,
                                          int use_part, Lds<TX>& lds) {
  // z-only CPML launches specialise their interior tiles; the all-axes kernel
  // keeps one general march (two would not fit its register budget)
  auto run = [&](const fd_tile& tl) {
    if constexpr (PM == 4) {
      if (!(tl.flags & FD_TILE_ZSLAB)) {
        run_tile<TX, PM, GAIN, false, NT>(tl, s, lds);
        return;
      }
    }
    run_tile<TX, PM, GAIN, (PM & 4) != 0, NT>(tl, s, lds);
  };
  if (use_part) {
    const int x = (int)blockIdx.x % 8, q = (int)blockIdx.x / 8;
    if (q < part.count[x]) {
      const fd_tile tl = tiles[part.start[x] + q];
      run(tl);
    }
    return;
  }
  for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
    const fd_tile tl = tiles[xcd_tile(w, ntiles)];
    run(tl);
  }
}

template <int TX, int PM, int GAIN, bool NT>
__global__ __launch_bounds__(FD_MAXBLOCK) void step_kernel(const fd_tile* __restrict__ tiles, int ntiles, int s,
                                                           fd_xcd part, int use_part) {
  __shared__ Lds<TX> lds;
  step_body<TX, PM, GAIN, NT>(tiles, ntiles, s, part, use_part, lds);
}

// All-axes CPML without gain: capped at four waves per SIMD (128 VGPRs; the
// compiler alone takes 134 and three waves), 7% faster on the beam box.
template <int TX, bool NT>
__global__ __launch_bounds__(FD_MAXBLOCK) __attribute__((amdgpu_waves_per_eu(4))) void step_kernel_ax(
    const fd_tile* __restrict__ tiles, int ntiles, int s, fd_xcd part, int use_part) {
  __shared__ Lds<TX> lds;
  step_body<TX, 7, 0, NT>(tiles, ntiles, s, part, use_part, lds);
}

// ------------------------------------------------------------- flux DFT
// Running DFT of the flux-plane fields (E^n at the plane, H^{n+1/2} averaged
// onto it), sampled every decim steps.  Samples go to a ring of FD_DFT_RING
// planes; the launch that takes the ring's last sample adds the whole ring to
// the FP64 accumulators, so each accumulator (16 bytes per point, component and
// frequency) is read and written once per ring rather than once per sample.
// The flush is a small dense product (samples x weights e^{i 2 pi f t_m});
// the weights of one frequency block are tabulated in LDS.

// Sample of component c (0 Ex, 1 Ey, 2 Hx, 3 Hy) at plane point p after step n.
__device__ __forceinline__ float dft_sample(const cdesc* d, int fl, int c, int p, long long n) {
  const int par = (int)(n & 1);
  const int kf = d->flux_k[fl];
  const int km = kf > 0 ? kf - 1 : d->nz - 1;
  if (c < 2) return G((const float*)d->E[par][c])[(size_t)kf * d->plane + p];
  const gf* h = G((const float*)d->H[par ^ 1][c - 2]);
  return 0.5f * (h[(size_t)km * d->plane + p] + h[(size_t)kf * d->plane + p]);
}

// complex product and integer power (square and multiply)
__device__ __forceinline__ void cmul(double ar, double ai, double br, double bi, double& cr, double& ci) {
  cr = ar * br - ai * bi;
  ci = ar * bi + ai * br;
}
__device__ __forceinline__ void cpow(double br, double bi, long long e, double& rr, double& ri) {
  rr = 1.0;
  ri = 0.0;
  while (e > 0) {
    if (e & 1) cmul(rr, ri, br, bi, rr, ri);
    cmul(br, bi, br, bi, br, bi);
    e >>= 1;
  }
}

// out = in + sum over the samples m < count (sample index first + m, step
// (first + m) decim) of v_m e^{i 2 pi f t_m} decim dt, for the work unit's
// FD_DFT_PTS points (one per lane), 4 components (one per wave) and FD_DFT_QB
// frequencies.  Sample m == fresh is taken from the fields after step nfresh
// instead of the ring.  first is a multiple of FD_DFT_RING; the weights are
// built from three unit phasors per frequency set up on the host (a ring, one
// sample and half a step of rotation): e^{i 2 pi f t_m} = R^(first/RING) S^m,
// and H samples carry the extra half step.
__device__ void dft_flush(const cdesc* d, int fl, int q0, int p0, long long first, int count, int fresh,
                          long long nfresh, const gd* in, gd* out, double (*tab)[FD_DFT_RING][4],
                          double (*base)[4], float (*samp)[FD_DFT_RING][64]) {
  const int nf = d->flux_nf[fl], plane = d->plane, decim = d->flux_decim[fl];
  const double dt = d->dt;
  const gd* rot = G((const double*)d->flux_rot[fl]);  // [nf][6]: R, S, half step
  if (threadIdx.x < FD_DFT_QB) {
    const int q = q0 + (int)threadIdx.x;
    double br = 1.0, bi = 0.0, hr = 1.0, hi = 0.0;
    if (q < nf) {
      cpow(rot[6 * q], rot[6 * q + 1], first / FD_DFT_RING, br, bi);
      hr = rot[6 * q + 4];
      hi = rot[6 * q + 5];
    }
    base[threadIdx.x][0] = br;
    base[threadIdx.x][1] = bi;
    base[threadIdx.x][2] = hr;
    base[threadIdx.x][3] = hi;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < FD_DFT_QB * FD_DFT_RING; idx += blockDim.x) {
    const int qq = idx / FD_DFT_RING, m = idx % FD_DFT_RING;
    const int q = q0 + qq;
    double ce = 0.0, se = 0.0, chh = 0.0, shh = 0.0;
    if (q < nf && m < count) {
      double sr, si;
      cpow(rot[6 * q + 2], rot[6 * q + 3], m, sr, si);
      const double* b0 = base[qq];
      cmul(b0[0], b0[1], sr, si, ce, se);
      cmul(ce, se, b0[2], b0[3], chh, shh);
    }
    tab[qq][m][0] = ce;
    tab[qq][m][1] = se;
    tab[qq][m][2] = chh;
    tab[qq][m][3] = shh;
  }
  __syncthreads();
  const gf* ring = G((const float*)d->flux_ring[fl]);
  const double w = (double)decim * dt;
  const int lane = threadIdx.x & 63;
  const int p = p0 + lane;
  if (p >= plane) return;
  const int wv = threadIdx.x >> 6;
  for (int c = wv; c < 4; c += blockDim.x >> 6) {  // one component per wave
    // the wave's samples go to LDS (8 loads in flight at a time); samples
    // m >= count have zero weight but must be finite
    float* sm = samp[wv][0];
    for (int m0 = 0; m0 < FD_DFT_RING; m0 += 8) {
      float v8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int m = m0 + u;
        v8[u] = ring[((size_t)(m < count ? m : 0) * 4 + c) * plane + p];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) sm[(m0 + u) * 64 + lane] = v8[u];
    }
    if (fresh >= 0) sm[fresh * 64 + lane] = dft_sample(d, fl, c, p, nfresh);
    // the block's sums, loaded ahead of the products
    const int nq = min(FD_DFT_QB, nf - q0);
    double ar[FD_DFT_QB], ai[FD_DFT_QB], re[FD_DFT_QB], im[FD_DFT_QB];
#pragma unroll
    for (int qq = 0; qq < FD_DFT_QB; ++qq) {
      const size_t at = 2 * (((size_t)c * nf + q0 + (qq < nq ? qq : 0)) * plane + p);
      ar[qq] = in[at];
      ai[qq] = in[at + 1];
      re[qq] = im[qq] = 0.0;
    }
    const int ph = c < 2 ? 0 : 2;
#pragma unroll 2
    for (int m = 0; m < FD_DFT_RING; ++m) {
      const double v = (double)sm[m * 64 + lane];
#pragma unroll
      for (int qq = 0; qq < FD_DFT_QB; ++qq) {
        re[qq] = fma(v, tab[qq][m][ph], re[qq]);
        im[qq] = fma(v, tab[qq][m][ph + 1], im[qq]);
      }
    }
#pragma unroll
    for (int qq = 0; qq < FD_DFT_QB; ++qq) {
      if (qq < nq) {
        const size_t at = 2 * (((size_t)c * nf + q0 + qq) * plane + p);
        out[at] = ar[qq] + re[qq] * w;
        out[at + 1] = ai[qq] + im[qq] * w;
      }
    }
  }
}

// In the step sequence: every decim steps of each realization, store the sample
// in its ring slot, or (last slot) add the ring and the sample to the sums.
__global__ __launch_bounds__(256) void dft_kernel(const fd_dft_tile* __restrict__ tiles, int s) {
  __shared__ double tab[FD_DFT_QB][FD_DFT_RING][4];
  const fd_dft_tile t = tiles[blockIdx.x];
  const cdesc* d = (const cdesc*)t.d;
  const int fl = t.flux;
  if (d->flux_nf[fl] == 0) return;
  const long long n = d->step + s;
  const int decim = d->flux_decim[fl];
  if (n % decim != 0) return;
  const long long si = n / decim;
  const int slot = (int)(si % FD_DFT_RING);
  if (slot < FD_DFT_RING - 1) {
    if (t.q0 != 0) return;
    const int plane = d->plane, p = t.p0 + (int)(threadIdx.x & 63);
    if (p >= plane) return;
    gf* ring = G(d->flux_ring[fl]);
    for (int c = threadIdx.x >> 6; c < 4; c += blockDim.x >> 6)
      ring[((size_t)slot * 4 + c) * plane + p] = dft_sample(d, fl, c, p, n);
    return;
  }
  __shared__ double base[FD_DFT_QB][4];
  __shared__ float samp[4][FD_DFT_RING][64];
  gd* acc = G(d->flux_acc[fl]);
  dft_flush(d, fl, t.q0, t.p0, si - (FD_DFT_RING - 1), FD_DFT_RING, FD_DFT_RING - 1, n, acc, acc, tab, base, samp);
}

// For reads: flux_prev = flux_acc + the count samples waiting in the ring
// (sample indices first ...), for flux plane fl; the sums themselves are kept.
__global__ __launch_bounds__(256) void dft_preview_kernel(const fd_dft_tile* __restrict__ tiles, int fl,
                                                          long long first, int count) {
  __shared__ double tab[FD_DFT_QB][FD_DFT_RING][4];
  const fd_dft_tile t = tiles[blockIdx.x];
  if (t.flux != fl) return;
  const cdesc* d = (const cdesc*)t.d;
  if (d->flux_nf[fl] == 0) return;
  __shared__ double base[FD_DFT_QB][4];
  __shared__ float samp[4][FD_DFT_RING][64];
  dft_flush(d, fl, t.q0, t.p0, first, count, -1, 0, G((const double*)d->flux_acc[fl]), G(d->flux_prev[fl]), tab,
            base, samp);
}

__global__ void advance_kernel(fd_desc* const* descs, int n, long long k) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) descs[t]->step += k;
}

__global__ void advance_one_kernel(fd_desc* d, long long k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) d->step += k;
}

__global__ void fill_kernel(uint4* p, size_t n16, uint8_t* tail, size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n16; q += stride)
    p[q] = make_uint4(0u, 0u, 0u, 0u);
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ntail) tail[t] = 0;
}

// Integer-exact voxelization: voxel centre X = (2 (i - origin) + 1) 2^16 quanta,
// inside sphere (C, rho) iff |X - C|^2 < rho^2 (minimum image on periodic axes).
// Candidate sites: those whose nominal position (h res 2^16 quanta along each axis)
// lies within `reach` of the voxel centre.
__device__ __forceinline__ long long floordiv_ll(long long a, long long b) {
  long long q = a / b;
  if ((a % b != 0) && (a < 0)) --q;
  return q;
}

__global__ void voxelize_kernel(const int64_t* __restrict__ sites, int ex, int ey, int ez, int3 per,
                                int3 ncr, int3 org, longlong3 reach, int res, int mat_bg, int mat_void,
                                int mat_out, int nx, int ny, int nz, int px, uint8_t* __restrict__ map) {
  const long long ncell = (long long)nx * ny * nz;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long H16 = 65536;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < ncell; v += stride) {
    const int i = (int)(v % nx);
    const int j = (int)((v / nx) % ny);
    const int k = (int)(v / ((long long)nx * ny));
    const int rel[3] = {i - org.x, j - org.y, k - org.z};
    const int nc[3] = {ncr.x, ncr.y, ncr.z};
    bool in_crystal = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) in_crystal = in_crystal && rel[a] >= 0 && rel[a] < nc[a];
    const long long vo = ((long long)k * ny + j) * px + i;  // padded rows
    if (!in_crystal) {
      map[vo] = (uint8_t)mat_out;
      continue;
    }
    const int pr[3] = {per.x, per.y, per.z};
    const long long rc[3] = {reach.x, reach.y, reach.z};
    const int ext[3] = {ex, ey, ez};
    const long long X[3] = {(2LL * rel[0] + 1) * H16, (2LL * rel[1] + 1) * H16, (2LL * rel[2] + 1) * H16};
    // res * 2^16 quanta between consecutive half-lattice sites; the period of a
    // periodic axis is the crystal length, ncr * 2^17 quanta
    long long hlo[3], hhi[3], sstep[3], period[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      sstep[a] = (long long)res * H16;
      period[a] = (long long)nc[a] * 2 * H16;
      hlo[a] = -floordiv_ll(-(X[a] - rc[a]), sstep[a]);  // ceil
      hhi[a] = floordiv_ll(X[a] + rc[a], sstep[a]);
      if (!pr[a]) {
        if (hlo[a] < 0) hlo[a] = 0;
        if (hhi[a] > ext[a] - 1) hhi[a] = ext[a] - 1;
      }
    }
    bool hit = false;
    for (long long l = hlo[2]; l <= hhi[2] && !hit; ++l) {
      long long lw = l;
      if (pr[2]) { lw %= ext[2]; if (lw < 0) lw += ext[2]; }
      for (long long kk = hlo[1]; kk <= hhi[1] && !hit; ++kk) {
        long long kw = kk;
        if (pr[1]) { kw %= ext[1]; if (kw < 0) kw += ext[1]; }
        for (long long h = hlo[0]; h <= hhi[0] && !hit; ++h) {
          long long hw = h;
          if (pr[0]) { hw %= ext[0]; if (hw < 0) hw += ext[0]; }
          if (((hw + kw + lw) & 1) != 0) continue;
          const int64_t* S = sites + 4 * ((lw * ey + kw) * ex + hw);
          const long long rho = S[3];
          if (rho <= 0) continue;
          long long r2 = 0;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            long long dd = X[a] - S[a];
            if (pr[a]) {
              dd %= period[a];
              if (dd < 0) dd += period[a];
              if (2 * dd > period[a]) dd -= period[a];
            }
            r2 += dd * dd;
          }
          if (r2 < rho * rho) hit = true;
        }
      }
    }
    map[vo] = (uint8_t)(hit ? mat_void : mat_bg);
  }
}

// Initial upper-level populations of the gain cells at their gain ordinals, as
// (hi, lo) pairs whose sum is n_init to about 48 bits (every other state
// variable starts at zero with the arena).
__global__ void init_pop_kernel(const uint8_t* __restrict__ map, const float* __restrict__ ninit,
                                const uint32_t* __restrict__ gidx, unsigned gainmask, float* pop, int ncell,
                                int nx, int px) {
  const int stride = gridDim.x * blockDim.x;
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < ncell; o += stride) {
    if (o % px >= nx) continue;  // row padding
    const int m = map[o];
    if (!((gainmask >> m) & 1u)) continue;
    const uint32_t g = gidx[o];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      pop[(size_t)q * ncell + g] = ninit[8 * m + 1 + q];        // hi
      pop[(size_t)(3 + q) * ncell + g] = ninit[8 * m + 5 + q];  // lo
    }
  }
}

// ------------------------------------- density matrix at the cell centres
// A density-matrix gain cell holds rho at its centre (i+1/2, j+1/2, k+1/2), where
// the paper solves the density-matrix equations.  The step kernels leave on
// every edge A = E^n + dt/(eps dx) (curl H - dx J_src), the field before the
// polarization change.  With <F> the average of the four edges of a component
// around a centre and [Q] on an edge a quarter of the sum of Q over the (up to
// four) gain cells sharing it -- the adjoint of <.>, so the field gives the
// matter exactly the energy the matter takes -- the matter then makes one
// predictor-corrector pass of the implicit midpoint coupling:
//   predictor  rho* = S(rho^n; <(E^n + A)/2>),   Q* = P(rho*) - P(rho^n) + dt J
//   corrector  E* = A - [Q*]/eps,  rho^{n+1} = S(rho^n; <(E^n + E*)/2>),
//              Q = P(rho^{n+1}) - P(rho^n) + dt J
//   edges      E^{n+1} = A - [Q]/eps
// with S = R(dt/2) C(E) R(dt/2), P_c = 2 kappa Re rho_0c, J the
// spontaneous-emission noise current at the centre and eps that of the edge's
// own voxel.  Each pass reads what the previous one wrote for neighbouring
// cells, so the passes are separate launches; a cell's rho is read and written
// only by its own thread.

// The plan's material table in LDS (a gain cell's own medium, an edge's
// permittivity), staged once per workgroup: a work unit's cells belong to one
// plan, so every coefficient read of the passes is an LDS read.
struct DmMats {
  fd_mat m[FD_MAXMAT];
};
__device__ __forceinline__ void dm_stage_mats(const cdesc* d, DmMats& sm) {
  const int words = d->nmat * (int)(sizeof(fd_mat) / 4);
  const gf* src = G((const float*)d->mats);
  float* dst = reinterpret_cast<float*>(sm.m);
  for (int q = (int)threadIdx.x; q < words; q += (int)blockDim.x) dst[q] = src[q];
  __syncthreads();
}

struct Ijk {
  int i, j, k;
};
__device__ __forceinline__ Ijk ijk_of(const cdesc* d, uint32_t o) {
  const uint32_t plane = (uint32_t)d->plane, px = (uint32_t)d->px;
  const uint32_t k = o / plane, r = o - k * plane, j = r / px;
  return {(int)(r - j * px), (int)j, (int)k};
}

// Coordinates of cell p's neighbours along each axis at offsets -1, 0, +1
// (periodic wrap; -1 beyond a PEC wall), so a cell's neighbourhood is indexed
// without divisions.
struct Nbr {
  int c[3][3];  // [axis][offset + 1]
};
__device__ __forceinline__ int wrap1(int i, int n, int per) {
  if (i >= 0 && i < n) return i;
  if (!per) return -1;
  return i < 0 ? i + n : i - n;
}
__device__ __forceinline__ Nbr neighbours(const cdesc* d, Ijk p) {
  Nbr b;
  const int q[3] = {p.i, p.j, p.k}, n[3] = {d->nx, d->ny, d->nz};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int o = 0; o < 3; ++o) b.c[a][o] = wrap1(q[a] + o - 1, n[a], d->per[a]);
  return b;
}
// The cell at offsets u, v in {-1, 0, 1} along the two axes transverse to
// component c ((c+1) mod 3, (c+2) mod 3), or -1 beyond a PEC wall; *held: the
// cell's component-c edge lies on a PEC wall (index 0 of a non-periodic
// transverse axis) and is held at zero.
__device__ __forceinline__ int nb_cell(const cdesc* d, const Nbr& b, int c, int u, int v, bool* held) {
  const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
  int o[3] = {1, 1, 1};
  o[a1] += u;
  o[a2] += v;
  const int x = b.c[0][o[0]], y = b.c[1][o[1]], z = b.c[2][o[2]];
  // bitwise, not short-circuit, operators: lane values must not become branches
  *held = ((!d->per[a1]) & (b.c[a1][o[a1]] == 0)) | ((!d->per[a2]) & (b.c[a2][o[a2]] == 0));
  return ((x | y | z) < 0) ? -1 : (z * d->ny + y) * d->px + x;
}

// A gain cell's state (populations as (hi, lo) FP32 pairs, coherences), its
// medium, its noise term dt J and P(rho^n).
struct DmCell {
  uint32_t g, o;
  Ijk p;
  const fd_mat* mt;
  float nh[3], nl[3], pp[3], inc[3];
  Cz c[3], x[3];
  float Pn[3], dJ[3];
};

__device__ __forceinline__ void dm_load(const cdesc* d, const DmMats& sm, uint32_t g, long long n, DmCell& z) {
  const size_t ncs = (size_t)d->ncell;
  const gf* pop = G((const float*)d->pop);
  z.g = g;
  z.o = ((const __attribute__((address_space(1))) uint32_t*)d->glist)[g];
  z.p = ijk_of(d, z.o);
  z.mt = &sm.m[((const gu8*)d->mat)[z.o]];
  const fd_mat& mt = *z.mt;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    z.nh[q] = pop[(size_t)q * ncs + g];
    z.nl[q] = pop[(size_t)(3 + q) * ncs + g];
    z.pp[q] = z.nh[q] + z.nl[q];
    z.inc[q] = 0.0f;
    z.c[q] = {pop[(size_t)(6 + q) * ncs + g], pop[(size_t)(9 + q) * ncs + g]};
    z.x[q] = {pop[(size_t)(12 + q) * ncs + g], pop[(size_t)(15 + q) * ncs + g]};
    z.Pn[q] = mt.bk2 * z.c[q].r;
    z.dJ[q] = 0.0f;
  }
  if (mt.noise != 0.0f) {
    float gg[3];
    // the counter takes the dense cell index (k ny + j) nx + i
    normals3((uint32_t)n, ((uint32_t)z.p.k * (uint32_t)d->ny + (uint32_t)z.p.j) * (uint32_t)d->nx + (uint32_t)z.p.i,
             d->key0, d->key1, gg);
#pragma unroll
    for (int q = 0; q < 3; ++q) z.dJ[q] = mt.noise * sqrtf(fmaxf(z.pp[q], 0.0f)) * gg[q];
  }
}

// Gathers are branch-free: an index beyond a PEC wall (-1) reads cell 0 and the
// value is replaced by 0 where it is used, so a thread's loads go out together
// and are waited for once (a load under a branch is waited for on its own).
__device__ __forceinline__ uint32_t clamp0(int e) { return e >= 0 ? (uint32_t)e : 0u; }

__global__ __launch_bounds__(FD_DM_CELLS) void dm_predict_kernel(const fd_dm_unit* __restrict__ units, int s) {
  __shared__ DmMats sm;
  const fd_dm_unit u = units[blockIdx.x];
  const cdesc* d = (const cdesc*)u.d;
  dm_stage_mats(d, sm);
  if ((int)threadIdx.x >= u.count) return;
  const long long n = d->step + s;
  const int par = (int)(n & 1);
  DmCell z;
  dm_load(d, sm, (uint32_t)(u.first + (int)threadIdx.x), n, z);
  const Nbr b = neighbours(d, z.p);
  float em[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    // <(E^n + A)/2>: the cell's four component-q edges sit at offsets {0, 1}
    const gf* En = G((const float*)d->E[par][q]);
    const gf* A = G((const float*)d->E[par ^ 1][q]);
    float acc = 0.0f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        bool held;
        const int e = nb_cell(d, b, q, a, c, &held);
        const uint32_t ec = clamp0(e);
        const float v = En[ec] + A[ec];
        acc += e >= 0 ? v : 0.0f;
      }
    em[q] = 0.125f * acc;
  }
  dm_relax(*z.mt, z.pp, z.inc, z.c, z.x);
  dm_cayley<false>(*z.mt, em, z.pp, z.inc, z.c, z.x);
  gf* Q = G(d->dmq[0]);
  const size_t ncs = (size_t)d->ncell;
#pragma unroll
  for (int q = 0; q < 3; ++q) Q[(size_t)q * ncs + z.o] = z.mt->bk2 * (z.c[q].r * z.mt->bf2) - z.Pn[q] + z.dJ[q];
}

__global__ __launch_bounds__(FD_DM_CELLS) void dm_correct_kernel(const fd_dm_unit* __restrict__ units, int s) {
  __shared__ DmMats sm;
  const fd_dm_unit u = units[blockIdx.x];
  const cdesc* d = (const cdesc*)u.d;
  dm_stage_mats(d, sm);
  if ((int)threadIdx.x >= u.count) return;
  const long long n = d->step + s;
  const int par = (int)(n & 1);
  DmCell z;
  dm_load(d, sm, (uint32_t)(u.first + (int)threadIdx.x), n, z);
  const Nbr b = neighbours(d, z.p);
  const gf* Qs = G((const float*)d->dmq[0]);
  const gu8* map = (const gu8*)d->mat;
  const size_t ncs = (size_t)d->ncell;
  float em[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    // Q* of the 3 x 3 cells around the centre across component q (0 off the
    // grid; cells without gain hold 0), and the voxels of the cell's four edges
    float qn[3][3];
    int ee[2][2];
    bool he[2][2];
    uint32_t me[2][2];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        bool held;
        const int e = nb_cell(d, b, q, a - 1, c - 1, &held);
        const float v = Qs[(size_t)q * ncs + clamp0(e)];
        qn[a][c] = e >= 0 ? v : 0.0f;
        if (a >= 1 && c >= 1) {
          ee[a - 1][c - 1] = e;
          he[a - 1][c - 1] = held;
          me[a - 1][c - 1] = map[clamp0(e)];
        }
      }
    // <E^n + E*> with E* = A - [Q*]/eps on the edges (0 beyond or on a PEC wall);
    // the edge at offsets (a, c) is shared by the cells at (a - 1 .. a, c - 1 .. c)
    const gf* En = G((const float*)d->E[par][q]);
    const gf* A = G((const float*)d->E[par ^ 1][q]);
    float acc = 0.0f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int e = ee[a][c];
        const uint32_t ec = clamp0(e);
        const float en = En[ec], av = A[ec];
        const float sh = 0.25f * ((qn[a][c] + qn[a + 1][c]) + (qn[a][c + 1] + qn[a + 1][c + 1]));
        const float es = av - sh * sm.m[me[a][c]].inv_eps;
        acc += e >= 0 ? en : 0.0f;
        acc += ((e >= 0) & !he[a][c]) ? es : 0.0f;
      }
    em[q] = 0.125f * acc;
  }
  dm_relax(*z.mt, z.pp, z.inc, z.c, z.x);
  dm_cayley<true>(*z.mt, em, z.pp, z.inc, z.c, z.x);
  dm_relax(*z.mt, z.pp, z.inc, z.c, z.x);
  gf* pop = G(d->pop);
  gf* Q = G(d->dmq[1]);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    Q[(size_t)r * ncs + z.o] = z.mt->bk2 * z.c[r].r - z.Pn[r] + z.dJ[r];
    two_sum(z.nh[r], z.nl[r], z.inc[r]);
    pop[(size_t)r * ncs + z.g] = z.nh[r];
    pop[(size_t)(3 + r) * ncs + z.g] = z.nl[r];
    pop[(size_t)(6 + r) * ncs + z.g] = z.c[r].r;
    pop[(size_t)(9 + r) * ncs + z.g] = z.c[r].i;
    pop[(size_t)(12 + r) * ncs + z.g] = z.x[r].r;
    pop[(size_t)(15 + r) * ncs + z.g] = z.x[r].i;
  }
}

// E^{n+1} = A - [Q]/eps on the edges next to gain cells, one listed cell per
// thread (the cells whose edges a gain cell shares): the twelve Q values first
// (cells without gain hold Q = 0), then, for a cell with a changed edge, its A
// and the new E.
__global__ __launch_bounds__(FD_DM_EDGES) void dm_edges_kernel(const fd_dm_unit* __restrict__ units, int s) {
  __shared__ DmMats sm;
  const fd_dm_unit u = units[blockIdx.x];
  const cdesc* d = (const cdesc*)u.d;
  dm_stage_mats(d, sm);
  const int t = (int)threadIdx.x;
  if (t >= u.count) return;
  const long long n = d->step + s;
  const int par = (int)(n & 1);
  const gf* Q = G((const float*)d->dmq[1]);
  const size_t ncs = (size_t)d->ncell;
  const uint32_t o = ((const __attribute__((address_space(1))) uint32_t*)d->elist)[u.first + t];
  const Nbr b = neighbours(d, ijk_of(d, o));
  // the cell's A and material go out with the sharers' Q (one round trip)
  float ev[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) ev[c] = G((const float*)d->E[par ^ 1][c])[o];
  const uint32_t mo = ((const gu8*)d->mat)[o];
  float acc[3];
  bool held[3];
  bool any = false;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    (void)nb_cell(d, b, c, 0, 0, &held[c]);
    // the cells sharing the edge: offsets {0, -1} along the transverse axes
    acc[c] = 0.0f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        bool h2;
        const int cc = nb_cell(d, b, c, -a, -v, &h2);
        const float qv = Q[(size_t)c * ncs + clamp0(cc)];
        acc[c] += cc >= 0 ? qv : 0.0f;
      }
    any = any | (!held[c] & (acc[c] != 0.0f));
  }
  if (!any) return;
  const float ie = sm.m[mo].inv_eps;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (!held[c] && acc[c] != 0.0f) G(d->E[par ^ 1][c])[o] = ev[c] - 0.25f * acc[c] * ie;
}

// After the edge pass: probe samples of E components and the T(t) partial of
// every xy tile of a flux plane, recomputed from the final E^{n+1} (the step
// kernels recorded them from A).  Unit: first = flux plane (-1: the probes),
// count = xy tile; the block has the plan's tile shape.
__global__ __launch_bounds__(FD_MAXBLOCK) void dm_diag_kernel(const fd_dm_unit* __restrict__ units, int s) {
  __shared__ double red[FD_MAXBLOCK / 64];
  const fd_dm_unit u = units[blockIdx.x];
  const cdesc* d = (const cdesc*)u.d;
  const long long n = d->step + s;
  const int par = (int)(n & 1);
  const int t = (int)threadIdx.x;
  if (u.first < 0) {
    if (t < d->nprobe && d->probe_comp[t] < 3)
      G(d->probe_ring)[(long long)t * d->max_steps + n] =
          G((const float*)d->E[par ^ 1][d->probe_comp[t]])[(size_t)d->probe_k[t] * d->plane + d->probe_cell[t]];
    return;
  }
  const int f = u.first, blk = u.count;
  const int TX = d->tile_x, TY = (int)blockDim.x / TX;
  const int ntx = (d->nx + TX - 1) / TX;
  const int i = (blk % ntx) * TX + t % TX, j = (blk / ntx) * TY + t / TX;
  double v = 0.0;
  if (i < d->nx && j < d->ny) {
    const int kf = d->flux_k[f], km = kf > 0 ? kf - 1 : d->nz - 1;
    const size_t off = (size_t)j * d->px + i;
    const size_t o = (size_t)kf * d->plane + off, om = (size_t)km * d->plane + off;
    const float sx = 0.5f * (G((const float*)d->E[par][0])[o] + G((const float*)d->E[par ^ 1][0])[o]);
    const float sy = 0.5f * (G((const float*)d->E[par][1])[o] + G((const float*)d->E[par ^ 1][1])[o]);
    const gf* hx = G((const float*)d->H[par ^ 1][0]);
    const gf* hy = G((const float*)d->H[par ^ 1][1]);
    const float hyc = 0.5f * (hy[om] + hy[o]), hxc = 0.5f * (hx[om] + hx[o]);
    v = (double)(sx * hyc) - (double)(sy * hxc);
  }
  const double tot = block_sum(v, red);
  if (t == 0) G(d->flux_T[f])[n * d->nblk + blk] = tot;
}

}  // namespace

// start/stop (optional) take the kernel's own begin and end timestamps
template <int TX, int PM, int GAIN>
static void launch_one(const fd_tile* tiles, int ntiles, int block, int grid, int s, const fd_xcd& part, int use,
                       int nt, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
  if constexpr (PM == 7 && GAIN == 0) {
    if (nt)
      hipExtLaunchKernelGGL(step_kernel_ax<TX, true>, dim3(grid), dim3(block), 0, st, start, stop, 0, tiles, ntiles,
                            s, part, use);
    else
      hipExtLaunchKernelGGL(step_kernel_ax<TX, false>, dim3(grid), dim3(block), 0, st, start, stop, 0, tiles, ntiles,
                            s, part, use);
  } else if (nt) {
    hipExtLaunchKernelGGL(step_kernel<TX, PM, GAIN, true>, dim3(grid), dim3(block), 0, st, start, stop, 0, tiles,
                          ntiles, s, part, use);
  } else {
    hipExtLaunchKernelGGL(step_kernel<TX, PM, GAIN, false>, dim3(grid), dim3(block), 0, st, start, stop, 0, tiles,
                          ntiles, s, part, use);
  }
}

template <int TX>
static hipError_t launch_tx(int cls, const fd_tile* tiles, int ntiles, int block, int grid, int s,
                            const fd_xcd& part, int use, int nt, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
  switch (cls) {
    case FD_CLASS_PLAIN: launch_one<TX, 0, 0>(tiles, ntiles, block, grid, s, part, use, nt, st, start, stop); break;
    case FD_CLASS_PMLZ: launch_one<TX, 4, 0>(tiles, ntiles, block, grid, s, part, use, nt, st, start, stop); break;
    case FD_CLASS_PML: launch_one<TX, 7, 0>(tiles, ntiles, block, grid, s, part, use, nt, st, start, stop); break;
    case FD_CLASS_GAIN: launch_one<TX, 0, 1>(tiles, ntiles, block, grid, s, part, use, nt, st, start, stop); break;
    case FD_CLASS_PMLZ_GAIN: launch_one<TX, 4, 1>(tiles, ntiles, block, grid, s, part, use, nt, st, start, stop); break;
    case FD_CLASS_PML_GAIN: launch_one<TX, 7, 1>(tiles, ntiles, block, grid, s, part, use, nt, st, start, stop); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t fd_launch_step(int cls, const fd_tile* tiles, int ntiles, int tile_x, int block, int grid, int s,
                          const fd_xcd* part, int nt, hipStream_t st, hipEvent_t start, hipEvent_t stop) {
  if (ntiles <= 0) return hipSuccess;
  if (block < 64 || block > FD_MAXBLOCK || (block & 63) != 0 || grid <= 0 || block % tile_x != 0 ||
      2 * (tile_x + 2) + 2 * (block / tile_x) > block)
    return hipErrorInvalidValue;
  fd_xcd pz{};
  int use = 0;
  if (part) {
    // every part must lie inside the list and the grid must cover the longest one
    int longest = 0;
    for (int x = 0; x < 8; ++x) {
      if (part->start[x] < 0 || part->count[x] < 0 || part->start[x] + part->count[x] > ntiles)
        return hipErrorInvalidValue;
      longest = part->count[x] > longest ? part->count[x] : longest;
    }
    if (grid < 8 * longest) return hipErrorInvalidValue;
    pz = *part;
    use = 1;
  }
  switch (tile_x) {
    case 16: return launch_tx<16>(cls, tiles, ntiles, block, grid, s, pz, use, nt, st, start, stop);
    case 32: return launch_tx<32>(cls, tiles, ntiles, block, grid, s, pz, use, nt, st, start, stop);
    case 64: return launch_tx<64>(cls, tiles, ntiles, block, grid, s, pz, use, nt, st, start, stop);
    default: return hipErrorInvalidValue;
  }
}

hipError_t fd_launch_dft(const fd_dft_tile* tiles, int ntiles, int s, hipStream_t st, hipEvent_t start,
                         hipEvent_t stop) {
  if (ntiles <= 0) return hipSuccess;
  hipExtLaunchKernelGGL(dft_kernel, dim3(ntiles), dim3(256), 0, st, start, stop, 0, tiles, s);
  return hipGetLastError();
}

hipError_t fd_launch_dft_preview(const fd_dft_tile* tiles, int ntiles, int flux, long long first, int count,
                                 hipStream_t st) {
  if (ntiles <= 0 || count <= 0) return hipSuccess;
  if (count > FD_DFT_RING || first < 0) return hipErrorInvalidValue;
  dft_preview_kernel<<<ntiles, 256, 0, st>>>(tiles, flux, first, count);
  return hipGetLastError();
}

hipError_t fd_launch_advance(fd_desc* const* descs, int n, long long k, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  advance_kernel<<<(n + 255) / 256, 256, 0, st>>>(descs, n, k);
  return hipGetLastError();
}

hipError_t fd_launch_advance_one(fd_desc* d, long long k, hipStream_t st) {
  advance_one_kernel<<<1, 64, 0, st>>>(d, k);
  return hipGetLastError();
}

hipError_t fd_launch_fill(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16;
  const size_t ntail = bytes - n16 * 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  fill_kernel<<<(unsigned)blocks, 256, 0, st>>>(reinterpret_cast<uint4*>(p), n16,
                                                reinterpret_cast<uint8_t*>(p) + n16 * 16, ntail);
  return hipGetLastError();
}

hipError_t fd_launch_voxelize(const int64_t* sites, int ex, int ey, int ez, const int* per, const int* ncr,
                              const int* origin, const int64_t* reach, int res, int mat_bg,
                              int mat_void, int mat_out, int nx, int ny, int nz, int px, uint8_t* map,
                              hipStream_t st) {
  const long long ncell = (long long)nx * ny * nz;
  long long blocks = (ncell + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  voxelize_kernel<<<(unsigned)blocks, 256, 0, st>>>(
      sites, ex, ey, ez, make_int3(per[0], per[1], per[2]), make_int3(ncr[0], ncr[1], ncr[2]),
      make_int3(origin[0], origin[1], origin[2]), make_longlong3(reach[0], reach[1], reach[2]), res, mat_bg,
      mat_void, mat_out, nx, ny, nz, px, map);
  return hipGetLastError();
}

hipError_t fd_launch_init_pop(const uint8_t* map, const float* n_init_by_mat, const uint32_t* gidx, unsigned gainmask,
                              float* pop, int ncell, int nx, int px, hipStream_t st) {
  int blocks = (ncell + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  init_pop_kernel<<<blocks, 256, 0, st>>>(map, n_init_by_mat, gidx, gainmask, pop, ncell, nx, px);
  return hipGetLastError();
}

// ------------------------------------------------------------ static tables
// The launch tables (tile lists, DFT work units, descriptor pointers) of batches
// made by fdtd_batch_create_static live here instead of in a hipMalloc'd block:
// one array per GPU, held until the process ends.  In host code the name is
// only a handle: kernels get the address hipGetSymbolAddress returns for the
// current device.
static __device__ __align__(256) unsigned char scratch[FD_STATIC_TABLE_BYTES];

hipError_t fd_static_tables(void** ptr, int* device) {
  static std::mutex mu;
  static void* addr[FD_MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= FD_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = a;
  }
  *ptr = addr[dev];
  *device = dev;
  return hipSuccess;
}

hipError_t fd_launch_dm(const fd_dm_unit* cells, int ncells, const fd_dm_unit* edges, int nedges,
                        const fd_dm_unit* diag, int ndiag, int block, int s, hipStream_t st, hipEvent_t* ev) {
  if (ncells <= 0) return hipSuccess;
  if (block < 64 || block > FD_MAXBLOCK || (block & 63) != 0) return hipErrorInvalidValue;
  auto E = [&](int q) -> hipEvent_t { return ev ? ev[q] : nullptr; };
  hipExtLaunchKernelGGL(dm_predict_kernel, dim3(ncells), dim3(FD_DM_CELLS), 0, st, E(0), E(1), 0, cells, s);
  hipExtLaunchKernelGGL(dm_correct_kernel, dim3(ncells), dim3(FD_DM_CELLS), 0, st, E(2), E(3), 0, cells, s);
  if (nedges > 0)
    hipExtLaunchKernelGGL(dm_edges_kernel, dim3(nedges), dim3(FD_DM_EDGES), 0, st, E(4), E(5), 0, edges, s);
  if (ndiag > 0) hipExtLaunchKernelGGL(dm_diag_kernel, dim3(ndiag), dim3(block), 0, st, E(6), E(7), 0, diag, s);
  return hipGetLastError();
}
