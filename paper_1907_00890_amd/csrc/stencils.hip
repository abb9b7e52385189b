// Marker-and-cell stencils around the Poisson solves (section 3.2: right-hand
// side of the split pressure equation and the velocity correction; section
// 3.6: the liquid-velocity extension and the interface velocity).
//
// Faces: u on i+1/2, v on j+1/2, w on k+1/2; a wall face (last index) has
// zero gradient, the face at -1/2 of a wall direction is implicit and zero.
// An outflow face (p = 0 on the face, half a cell beyond the centre) is
// handled through a mirrored ghost cell: p, p_hat and phi of the ghost are
// minus the end cell's, rho is the end cell's, at distance dz of the end
// cell (the plan stores it as the last centre distance).  The face stencils
// take such faces at upper ends (the last stored face of a direction); the
// residual (the Laplacian alone) takes them at any end.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace vp {

// ---------------------------------------------------------------------------
// Launch geometry shared by the stencils: a block is a TX x TY tile of one
// z-plane (TX = min(nx, 64), 256 threads) and marches through `kc`
// consecutive planes, keeping the values at k-1, k, k+1 of the fields that
// are read at z-neighbours in registers.  x and y neighbours are re-read
// through L1 (they are loaded by the same block, except the tile's halo).
// The 7-point kernels (right-hand side, residual) march a few planes; the
// streaming ones (correction, extension) take one plane per block.
// ---------------------------------------------------------------------------
struct Tile {
  int i, j, kb, ke;
  bool ok;
  long c0;     // offset of (i, j, 0)
  long xp, xm, yp, ym;  // in-plane neighbour offsets (wrapped: valid cells also at walls)
  bool hxp, hxm, hyp, hym;
};

// Tile width: the largest power of two dividing nx, at most TXMAX (64 for
// the marching 7-point kernels: taller tiles, fewer halo rows; 256 for the
// streaming ones: whole rows of power-of-two grids).
template <int TXMAX>
__host__ __device__ __forceinline__ int tile_w(const GridArgs& g) {
  return g.txp < TXMAX ? g.txp : TXMAX;
}

template <int TXMAX>
__device__ __forceinline__ Tile tile_of(const GridArgs& g) {
  Tile t;
  const int tx = tile_w<TXMAX>(g);
  const int ltx = __builtin_ctz(tx);
  t.i = blockIdx.x * tx + (threadIdx.x & (tx - 1));
  t.j = blockIdx.y * (256 / tx) + (threadIdx.x >> ltx);
  t.kb = blockIdx.z * g.kc;
  t.ke = t.kb + g.kc < g.nz ? t.kb + g.kc : g.nz;
  t.ok = t.j < g.ny;
  t.c0 = (long)t.j * g.nx + t.i;
  t.hxp = t.i + 1 < g.nx || g.bcx == 0;
  t.hxm = t.i > 0 || g.bcx == 0;
  t.hyp = t.j + 1 < g.ny || g.bcy == 0;
  t.hym = t.j > 0 || g.bcy == 0;
  t.xp = t.i + 1 < g.nx ? 1 : -(long)(g.nx - 1);
  t.xm = t.i > 0 ? -1 : (long)(g.nx - 1);
  t.yp = t.j + 1 < g.ny ? (long)g.nx : -(long)(g.ny - 1) * g.nx;
  t.ym = t.j > 0 ? -(long)g.nx : (long)(g.ny - 1) * g.nx;
  return t;
}

// plane index of the z-neighbours of plane k; -1 at a wall
__device__ __forceinline__ int kplus(const GridArgs& g, int k) {
  return k + 1 < g.nz ? k + 1 : (g.bcz == 0 ? 0 : -1);
}
__device__ __forceinline__ int kminus(const GridArgs& g, int k) {
  return k > 0 ? k - 1 : (g.bcz == 0 ? g.nz - 1 : -1);
}

// the upper z-face of plane k is an outflow face
__device__ __forceinline__ bool ztop_out(const GridArgs& g, int k) {
  return k == g.nz - 1 && (g.outflow & 32);
}
// outflow at the upper x / y end (the face of the cell with the last index)
__device__ __forceinline__ bool xtop_out(const GridArgs& g) { return (g.outflow & 2) != 0; }
__device__ __forceinline__ bool ytop_out(const GridArgs& g) { return (g.outflow & 8) != 0; }

// inverse of the face density 1 / ((rho_a + rho_b) / 2) (densities > 0)
__device__ __forceinline__ double inv_face_rho(double ra, double rb) {
  return 2.0 * rcp64(ra + rb);
}

// One cell of the split right-hand side from its neighbourhood, with the
// inverse z widths (1/dzc of the upper and lower faces, 1/dzf) passed in:
// the divisions of the stencil become multiplications and the face
// densities take the refined hardware reciprocal (measured at 256^3: 205 ->
// 191 us; within an ulp or two of IEEE division).  Floating-point
// contraction is off inside, so every kernel variant that calls it (plain or
// LDS-staged tiles) produces the same bits.  The neighbour values of a face
// that does not exist (wall) are not used.
struct RhsNbr {
  double ph, rh;  // p_hat and rho across the face
  bool has;       // the face is not a wall
};
__device__ __forceinline__ double rhs_cell(double rho0, double ir0, double idx, double idy,
                                           double r0dt, double phc, double rhc, RhsNbr xp,
                                           RhsNbr xm, RhsNbr yp, RhsNbr ym, RhsNbr zp, double idzcp,
                                           RhsNbr zm, double idzcm, double idzf, double uc,
                                           double um, double vc, double vm, double wc, double wm,
                                           double sv) {
#pragma clang fp contract(off)
  double fxp = 0.0, fxm = 0.0, fyp = 0.0, fym = 0.0, fzp = 0.0, fzm = 0.0;
  if (xp.has) fxp = (ir0 - inv_face_rho(rhc, xp.rh)) * (xp.ph - phc) * idx;
  if (xm.has) fxm = (ir0 - inv_face_rho(xm.rh, rhc)) * (phc - xm.ph) * idx;
  if (yp.has) fyp = (ir0 - inv_face_rho(rhc, yp.rh)) * (yp.ph - phc) * idy;
  if (ym.has) fym = (ir0 - inv_face_rho(ym.rh, rhc)) * (phc - ym.ph) * idy;
  if (zp.has) fzp = (ir0 - inv_face_rho(rhc, zp.rh)) * (zp.ph - phc) * idzcp;
  if (zm.has) fzm = (ir0 - inv_face_rho(zm.rh, rhc)) * (phc - zm.ph) * idzcm;
  const double divf = (fxp - fxm) * idx + (fyp - fym) * idy + (fzp - fzm) * idzf;
  const double divu = (uc - um) * idx + (vc - vm) * idy + (wc - (zm.has ? wm : 0.0)) * idzf;
  return rho0 * divf + r0dt * (divu - sv);
}

// b = rho0 D[(1/rho0 - 1/rho_f) G p_hat] + (rho0/dt) (D u* - s)
__global__ __launch_bounds__(256) void k_rhs(const GridArgs g, const double* __restrict__ u,
                                              const double* __restrict__ v,
                                              const double* __restrict__ w,
                                              const double* __restrict__ ph,
                                              const double* __restrict__ rho, double rho0,
                                              const double* __restrict__ src, double dt,
                                              double* __restrict__ b) {
  const Tile t = tile_of<64>(g);
  if (!t.ok) return;
  const long P = (long)g.nx * g.ny;
  const double ir0 = 1.0 / rho0, idx = 1.0 / g.dx, idy = 1.0 / g.dy, r0dt = rho0 / dt;
  int km = kminus(g, t.kb);
  double phm = 0.0, rhm = 0.0, wm = 0.0;
  if (km >= 0) {
    phm = ph[km * P + t.c0];
    rhm = rho[km * P + t.c0];
    wm = w[km * P + t.c0];
  }
  double phc = ph[t.kb * P + t.c0], rhc = rho[t.kb * P + t.c0];
  for (int k = t.kb; k < t.ke; ++k) {
    const long c = k * P + t.c0;
    const int kp = kplus(g, k);
    const bool zph = kp >= 0 || ztop_out(g, k);
    double php = 0.0, rhp = 0.0;
    if (kp >= 0) {
      php = ph[kp * P + t.c0];
      rhp = rho[kp * P + t.c0];
    } else if (zph) {
      php = -phc;
      rhp = rhc;
    }
    const RhsNbr xp = t.hxp ? RhsNbr{ph[c + t.xp], rho[c + t.xp], true}
                            : RhsNbr{-phc, rhc, xtop_out(g)};
    const RhsNbr xm{t.hxm ? ph[c + t.xm] : 0.0, t.hxm ? rho[c + t.xm] : 0.0, t.hxm};
    const RhsNbr yp = t.hyp ? RhsNbr{ph[c + t.yp], rho[c + t.yp], true}
                            : RhsNbr{-phc, rhc, ytop_out(g)};
    const RhsNbr ym{t.hym ? ph[c + t.ym] : 0.0, t.hym ? rho[c + t.ym] : 0.0, t.hym};
    const RhsNbr zp{php, rhp, zph}, zm{phm, rhm, km >= 0};
    const double wc = w[c];
    const double um = t.hxm ? u[c + t.xm] : 0.0;
    const double vm = t.hym ? v[c + t.ym] : 0.0;
    const double sv = src ? src[c] : 0.0;
    b[c] = rhs_cell(rho0, ir0, idx, idy, r0dt, phc, rhc, xp, xm, yp, ym, zp,
                    zph ? 1.0 / g.dzc[k] : 1.0, zm, km >= 0 ? 1.0 / g.dzc[km] : 1.0,
                    1.0 / g.dzf[k], u[c], um,
                    v[c], vm, wc, wm, sv);
    phm = phc; phc = php;
    rhm = rhc; rhc = rhp;
    wm = wc;
    km = k;
  }
}

// The same right-hand side on 64 x TY tiles (TY = 8 or 16; nx % 64 == 0,
// ny % TY == 0):
// p_hat and rho of the current plane, with their x and y halo, are staged in
// LDS once per block and plane, and their z-neighbours stay in registers
// while the block marches through its planes, so every value of the two
// 7-point fields is read from HBM about once (halo: 2/TY rows, 2/64 columns,
// 2/kc planes).  A thread owns column tx of rows ty, ty+4, ... of the tile.
// The loads of plane k+1 are issued before plane k is computed, into the
// other of two register sets (steps alternate between them, so no register
// is copied while its load is in flight).  Every load is unconditional (at a
// wall, or for a thread without a halo cell, the address is a valid cell
// whose value is not used; without s the u* stream stands in), so the
// compiler counts the outstanding memory operations exactly and waits only
// for the plane it computes.  w* and s, read by one cell each, are loaded
// non-temporally, and b is stored so (measured at 256^3: 210 -> 205 us).
// The per-cell arithmetic is k_rhs's, term for term.
template <int TY>
__global__ __launch_bounds__(256) void k_rhs_tiled(
    const GridArgs g, const double* __restrict__ u, const double* __restrict__ v,
    const double* __restrict__ w, const double* __restrict__ ph, const double* __restrict__ rho,
    double rho0, const double* __restrict__ src, double dt, const double* __restrict__ dzf,
    const double* __restrict__ dzc, double* __restrict__ b) {
  constexpr int TX = 64, W = TX + 2, RPT = TY / 4;
  __shared__ double sph[(TY + 2) * W], srh[(TY + 2) * W];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
  const int kb = blockIdx.z * g.kc, ke = kb + g.kc < g.nz ? kb + g.kc : g.nz;
  const int i = i0 + tx;
  const long P = (long)g.nx * g.ny;
  const double ir0 = 1.0 / rho0, idx = 1.0 / g.dx, idy = 1.0 / g.dy, r0dt = rho0 / dt;
  const bool hxp = i + 1 < g.nx || g.bcx == 0, hxm = i > 0 || g.bcx == 0;
  const long xm = i > 0 ? -1 : (long)(g.nx - 1);
  const bool has_src = src != nullptr;
  const double* sp = has_src ? src : u;
  // halo cell h of this plane (threads 0 .. 2*TY + 2*TX - 1): LDS slot and
  // in-plane offset; wrapped when periodic, clamped (and unused) at walls
  int hslot = -1;
  long hoff = 0;
  {
    const int h = threadIdx.x;
    int r = 0, c = 0;
    if (h < 2 * TY) {
      r = h % TY;
      c = h < TY ? -1 : TX;
    } else if (h < 2 * TY + 2 * TX) {
      c = (h - 2 * TY) % TX;
      r = h - 2 * TY < TX ? -1 : TY;
    }
    if (h < 2 * TY + 2 * TX) {
      int gi = i0 + c, gj = j0 + r;
      if (gi < 0) gi = g.bcx == 0 ? g.nx - 1 : 0;
      if (gi >= g.nx) gi = g.bcx == 0 ? 0 : g.nx - 1;
      if (gj < 0) gj = g.bcy == 0 ? g.ny - 1 : 0;
      if (gj >= g.ny) gj = g.bcy == 0 ? 0 : g.ny - 1;
      hslot = (r + 1) * W + (c + 1);
      hoff = (long)gj * g.nx + gi;
    }
  }
  long c0[RPT];
  bool hyp[RPT], hym[RPT];
  long ymo[RPT];
  double phm[RPT], phc[RPT], rhm[RPT], rhc[RPT], wm[RPT];
  int km = kminus(g, kb);
#pragma unroll
  for (int m = 0; m < RPT; ++m) {
    const int j = j0 + ty + 4 * m;
    c0[m] = (long)j * g.nx + i;
    hyp[m] = j + 1 < g.ny || g.bcy == 0;
    hym[m] = j > 0 || g.bcy == 0;
    ymo[m] = j > 0 ? -(long)g.nx : (long)(g.ny - 1) * g.nx;
    phm[m] = rhm[m] = wm[m] = 0.0;
    if (km >= 0) {
      phm[m] = ph[km * P + c0[m]];
      rhm[m] = rho[km * P + c0[m]];
      wm[m] = w[km * P + c0[m]];
    }
    phc[m] = ph[kb * P + c0[m]];
    rhc[m] = rho[kb * P + c0[m]];
  }
  // the loads of one plane k: the z+1 neighbours of p_hat and rho (plane k
  // itself at a wall), u* and v* with their x- / y- neighbours, w*, s, and
  // this thread's halo cell of p_hat and rho
  struct PlaneLoads {
    double php[RPT], rhp[RPT], uc[RPT], um[RPT], vc[RPT], vm[RPT], wc[RPT], sv[RPT], hph, hrh;
  };
  auto issue = [&](int k, PlaneLoads& L) {
    const int kp = kplus(g, k);
    const long ko = (long)k * P, kpo = (long)(kp >= 0 ? kp : k) * P;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      L.php[m] = ph[kpo + c0[m]];
      L.rhp[m] = rho[kpo + c0[m]];
      L.uc[m] = u[ko + c0[m]];
      L.um[m] = u[ko + c0[m] + xm];
      L.vc[m] = v[ko + c0[m]];
      L.vm[m] = v[ko + c0[m] + ymo[m]];
      L.wc[m] = __builtin_nontemporal_load(w + ko + c0[m]);
      L.sv[m] = __builtin_nontemporal_load(sp + ko + c0[m]);
    }
    L.hph = ph[ko + hoff];
    L.hrh = rho[ko + hoff];
  };
  // plane k from the loads L; with `pref`, plane k+1's loads go into Ln first
  auto step = [&](int k, PlaneLoads& L, PlaneLoads& Ln, auto pref_c) {
    if constexpr (decltype(pref_c)::value) issue(k + 1, Ln);
    const int kp = kplus(g, k);
    const bool zph = kp >= 0 || ztop_out(g, k);
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const int slot = (ty + 4 * m + 1) * W + tx + 1;
      sph[slot] = phc[m];
      srh[slot] = rhc[m];
    }
    if (hslot >= 0) {
      sph[hslot] = L.hph;
      srh[hslot] = L.hrh;
    }
    __syncthreads();
    const double idzf = 1.0 / dzf[k];
    const double idzcp = zph ? 1.0 / dzc[k] : 1.0, idzcm = km >= 0 ? 1.0 / dzc[km] : 1.0;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const long c = k * P + c0[m];
      const int sl = (ty + 4 * m + 1) * W + tx + 1;
      double php = 0.0, rhp = 0.0;
      if (kp >= 0) {
        php = L.php[m];
        rhp = L.rhp[m];
      } else if (zph) {
        php = -phc[m];
        rhp = rhc[m];
      }
      const RhsNbr xp = hxp ? RhsNbr{sph[sl + 1], srh[sl + 1], true}
                            : RhsNbr{-phc[m], rhc[m], xtop_out(g)};
      const RhsNbr xmn{sph[sl - 1], srh[sl - 1], hxm};
      const RhsNbr yp = hyp[m] ? RhsNbr{sph[sl + W], srh[sl + W], true}
                               : RhsNbr{-phc[m], rhc[m], ytop_out(g)};
      const RhsNbr ym{sph[sl - W], srh[sl - W], hym[m]};
      const RhsNbr zp{php, rhp, zph}, zm{phm[m], rhm[m], km >= 0};
      const double wc = L.wc[m];
      __builtin_nontemporal_store(
          rhs_cell(rho0, ir0, idx, idy, r0dt, phc[m], rhc[m], xp, xmn, yp, ym, zp, idzcp, zm,
                   idzcm, idzf, L.uc[m], hxm ? L.um[m] : 0.0, L.vc[m], hym[m] ? L.vm[m] : 0.0, wc, wm[m],
                   has_src ? L.sv[m] : 0.0),
          b + c);
      phm[m] = phc[m];
      phc[m] = php;
      rhm[m] = rhc[m];
      rhc[m] = rhp;
      wm[m] = wc;
    }
    km = k;
    __syncthreads();  // the tile is rewritten for the next plane
  };
  using F = std::false_type;
  using T = std::true_type;
  PlaneLoads la, lb;
  issue(kb, la);
  int k = kb;
  for (; k + 2 < ke; k += 2) {
    step(k, la, lb, T{});
    step(k + 1, lb, la, T{});
  }
  if (k + 1 < ke) {
    step(k, la, lb, T{});
    step(k + 1, lb, la, F{});
  } else {
    step(k, la, lb, F{});
  }
}

// One "+" face of the fused epilogue: the corrected velocity from u* and the
// jumps of p, p_hat, rho and phi across the face (hinv = 1/dx, 1/dy or the
// inverse centre distance 1/dzc), and the gradient of phi through *gphi.
// Contraction is off inside: every kernel variant gives the same bits.
__device__ __forceinline__ double epi_face(double un, double dt, double ir0, double pn, double pc,
                                           double rn, double rc, double hn, double hc, double fn,
                                           double fc, double hinv, double* gphi) {
#pragma clang fp contract(off)
  *gphi = (fn - fc) * hinv;
  return un - dt * (ir0 * (pn - pc) * hinv + (inv_face_rho(rc, rn) - ir0) * (hn - hc) * hinv);
}

// u <- u* - dt [ (1/rho0) G p + (1/rho_f - 1/rho0) G p_hat ] on the cell's
// three "plus" faces (epi_face's arithmetic: the LDS-tiled variant, the
// epilogue's correction kind, gives the same bits)
__global__ __launch_bounds__(256) void k_correct(const GridArgs g, double* __restrict__ u,
                                                  double* __restrict__ v, double* __restrict__ w,
                                                  const double* __restrict__ p,
                                                  const double* __restrict__ ph,
                                                  const double* __restrict__ rho, double rho0,
                                                  double dt) {
  const Tile t = tile_of<256>(g);
  if (!t.ok) return;
  const long P = (long)g.nx * g.ny;
  const double ir0 = 1.0 / rho0, idx = 1.0 / g.dx, idy = 1.0 / g.dy;
  double pc = p[t.kb * P + t.c0], hc = ph[t.kb * P + t.c0], rc = rho[t.kb * P + t.c0];
  for (int k = t.kb; k < t.ke; ++k) {
    const long c = k * P + t.c0;
    const int kp = kplus(g, k);
    const bool zph = kp >= 0 || ztop_out(g, k);
    double pp = 0.0, hp = 0.0, rp = 0.0;
    if (kp >= 0) {
      pp = p[kp * P + t.c0];
      hp = ph[kp * P + t.c0];
      rp = rho[kp * P + t.c0];
    } else if (zph) {
      pp = -pc;
      hp = -hc;
      rp = rc;
    }
    double gnone;  // epi_face's phi gradient, unused here (no phi)
    if (t.hxp || xtop_out(g)) {
      const double pn = t.hxp ? p[c + t.xp] : -pc, hn = t.hxp ? ph[c + t.xp] : -hc;
      const double rn = t.hxp ? rho[c + t.xp] : rc;
      __builtin_nontemporal_store(
          epi_face(u[c], dt, ir0, pn, pc, rn, rc, hn, hc, 0.0, 0.0, idx, &gnone), u + c);
    }
    if (t.hyp || ytop_out(g)) {
      const double pn = t.hyp ? p[c + t.yp] : -pc, hn = t.hyp ? ph[c + t.yp] : -hc;
      const double rn = t.hyp ? rho[c + t.yp] : rc;
      __builtin_nontemporal_store(
          epi_face(v[c], dt, ir0, pn, pc, rn, rc, hn, hc, 0.0, 0.0, idy, &gnone), v + c);
    }
    if (zph)
      __builtin_nontemporal_store(
          epi_face(w[c], dt, ir0, pp, pc, rp, rc, hp, hc, 0.0, 0.0, 1.0 / g.dzc[k], &gnone),
          w + c);
    pc = pp;
    hc = hp;
    rc = rp;
  }
}

// u_1^e = u - G phi ; u_Gamma = u_1^e - q (the differences of epi_face, as
// the LDS-tiled variant takes them)
__global__ __launch_bounds__(256) void k_extend(const GridArgs g, const double* __restrict__ u,
                                                 const double* __restrict__ v,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ phi,
                                                 const double* __restrict__ qx,
                                                 const double* __restrict__ qy,
                                                 const double* __restrict__ qz,
                                                 double* __restrict__ ue, double* __restrict__ ve,
                                                 double* __restrict__ we, double* __restrict__ ug,
                                                 double* __restrict__ vg, double* __restrict__ wg) {
  const Tile t = tile_of<256>(g);
  if (!t.ok) return;
  const long P = (long)g.nx * g.ny;
  const double idx = 1.0 / g.dx, idy = 1.0 / g.dy;
  double fc = phi[t.kb * P + t.c0];
  for (int k = t.kb; k < t.ke; ++k) {
    const long c = k * P + t.c0;
    const int kp = kplus(g, k);
    const bool zph = kp >= 0 || ztop_out(g, k);
    const double fp = kp >= 0 ? phi[kp * P + t.c0] : (zph ? -fc : 0.0);
    const double gx = t.hxp ? (phi[c + t.xp] - fc) * idx : (xtop_out(g) ? (-fc - fc) * idx : 0.0);
    const double gy = t.hyp ? (phi[c + t.yp] - fc) * idy : (ytop_out(g) ? (-fc - fc) * idy : 0.0);
    const double gz = zph ? (fp - fc) * (1.0 / g.dzc[k]) : 0.0;
    const double a = u[c] - gx, bb = v[c] - gy, cc = w[c] - gz;
    __builtin_nontemporal_store(a, ue + c);
    __builtin_nontemporal_store(bb, ve + c);
    __builtin_nontemporal_store(cc, we + c);
    if (ug) {
      __builtin_nontemporal_store(a - qx[c], ug + c);
      __builtin_nontemporal_store(bb - qy[c], vg + c);
      __builtin_nontemporal_store(cc - qz[c], wg + c);
    }
    fc = fp;
  }
}

__device__ __forceinline__ void epi_store(double un, double vn, double wn, double gx, double gy,
                                          double gz, long c, double* __restrict__ u,
                                          double* __restrict__ v, double* __restrict__ w,
                                          const double* __restrict__ qx,
                                          const double* __restrict__ qy,
                                          const double* __restrict__ qz, double qxv, double qyv,
                                          double qzv, bool have_q, double* __restrict__ ue,
                                          double* __restrict__ ve, double* __restrict__ we,
                                          double* __restrict__ ug, double* __restrict__ vg,
                                          double* __restrict__ wg) {
#pragma clang fp contract(off)
  // the outputs are not read again by this kernel: non-temporal stores
  __builtin_nontemporal_store(un, u + c);
  __builtin_nontemporal_store(vn, v + c);
  __builtin_nontemporal_store(wn, w + c);
  const double ex = un - gx, ey = vn - gy, ez = wn - gz;
  if (ue) {
    __builtin_nontemporal_store(ex, ue + c);
    __builtin_nontemporal_store(ey, ve + c);
    __builtin_nontemporal_store(ez, we + c);
  }
  if (ug) {
    __builtin_nontemporal_store(ex - (have_q ? qxv : qx[c]), ug + c);
    __builtin_nontemporal_store(ey - (have_q ? qyv : qy[c]), vg + c);
    __builtin_nontemporal_store(ez - (have_q ? qzv : qz[c]), wg + c);
  }
}

// One time step's two stencils after the solves, fused: on each of the
// cell's "+" faces
//   u^{n+1} = u* - dt [ (1/rho0) G p + (1/rho_f - 1/rho0) G p_hat ]  (in place)
//   u_1^e   = u^{n+1} - G phi,   u_Gamma = u_1^e - q
__global__ __launch_bounds__(256) void k_step_epilogue(
    const GridArgs g, double* __restrict__ u, double* __restrict__ v, double* __restrict__ w,
    const double* __restrict__ p, const double* __restrict__ ph, const double* __restrict__ rho,
    double rho0, double dt, const double* __restrict__ phi, const double* __restrict__ qx,
    const double* __restrict__ qy, const double* __restrict__ qz, double* __restrict__ ue,
    double* __restrict__ ve, double* __restrict__ we, double* __restrict__ ug,
    double* __restrict__ vg, double* __restrict__ wg) {
  const Tile t = tile_of<256>(g);
  if (!t.ok) return;
  const long P = (long)g.nx * g.ny;
  const double ir0 = 1.0 / rho0, idx = 1.0 / g.dx, idy = 1.0 / g.dy;
  // the z-neighbour values of plane k become the centre values of plane k+1
  double pc = p[t.kb * P + t.c0], hc = ph[t.kb * P + t.c0], rc = rho[t.kb * P + t.c0],
         fc = phi[t.kb * P + t.c0];
  for (int k = t.kb; k < t.ke; ++k) {
    const long c = k * P + t.c0;
    const int kp = kplus(g, k);
    double un = u[c], vn = v[c], wn = w[c];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    if (t.hxp) {
      const long n = c + t.xp;
      un = epi_face(un, dt, ir0, p[n], pc, rho[n], rc, ph[n], hc, phi[n], fc, idx, &gx);
    } else if (xtop_out(g)) {
      un = epi_face(un, dt, ir0, -pc, pc, rc, rc, -hc, hc, -fc, fc, idx, &gx);
    }
    if (t.hyp) {
      const long n = c + t.yp;
      vn = epi_face(vn, dt, ir0, p[n], pc, rho[n], rc, ph[n], hc, phi[n], fc, idy, &gy);
    } else if (ytop_out(g)) {
      vn = epi_face(vn, dt, ir0, -pc, pc, rc, rc, -hc, hc, -fc, fc, idy, &gy);
    }
    double pp = 0.0, hp = 0.0, rp = 0.0, fp = 0.0;
    const bool zph = kp >= 0 || ztop_out(g, k);
    if (kp >= 0) {
      const long n = kp * P + t.c0;
      pp = p[n];
      hp = ph[n];
      rp = rho[n];
      fp = phi[n];
    } else if (zph) {
      pp = -pc;
      hp = -hc;
      rp = rc;
      fp = -fc;
    }
    if (zph) wn = epi_face(wn, dt, ir0, pp, pc, rp, rc, hp, hc, fp, fc, 1.0 / g.dzc[k], &gz);
    epi_store(un, vn, wn, gx, gy, gz, c, u, v, w, qx, qy, qz, 0.0, 0.0, 0.0, false, ue, ve, we, ug,
              vg, wg);
    pc = pp;
    hc = hp;
    rc = rp;
    fc = fp;
  }
}

// The fused epilogue on 64 x TY tiles (nx % 64 == 0, ny % TY == 0), marching
// g.kc planes: p, p_hat, rho and phi of the current plane, with their +x and
// +y halo, are staged in LDS once per block and plane, and their +z values
// (the next plane's centre values) stay in registers, so each of these four
// fields is read from HBM about once.  All loads of a plane are issued
// before its barrier.  Blocks take the tile rows and plane chunks last
// first: the x inverse before it writes p and phi in row order, so the last
// rows are the likeliest to still sit in the Infinity Cache (measured at
// 256^3: 487 -> 479 us).  The per-face arithmetic is k_step_epilogue's.
// KIND: EPI_STEP (the fused epilogue), EPI_CORRECT (the correction alone:
// p, p_hat, rho staged; u, v, w updated in place, nothing else written) or
// EPI_EXTEND (the extension alone: phi staged; u, v, w read, ue.. and, with q,
// ug.. written).
enum : int { EPI_STEP = 0, EPI_CORRECT = 1, EPI_EXTEND = 2 };

template <int TY, int KIND>
__global__ __launch_bounds__(256) void k_step_epilogue_tiled(
    const GridArgs g, double* __restrict__ u, double* __restrict__ v, double* __restrict__ w,
    const double* __restrict__ p, const double* __restrict__ ph, const double* __restrict__ rho,
    double rho0, double dt, const double* __restrict__ phi, const double* __restrict__ qx,
    const double* __restrict__ qy, const double* __restrict__ qz, double* __restrict__ ue,
    double* __restrict__ ve, double* __restrict__ we, double* __restrict__ ug,
    double* __restrict__ vg, double* __restrict__ wg) {
  constexpr int TX = 64, W = TX + 1, RPT = TY / 4, AREA = (TY + 1) * W;
  constexpr bool PHR = KIND != EPI_EXTEND, PHI = KIND != EPI_CORRECT;  // fields staged
  __shared__ double sm[4 * AREA];  // p, p_hat, rho, phi
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int by = gridDim.y - 1 - blockIdx.y, bz = gridDim.z - 1 - blockIdx.z;  // last first
  const int i0 = blockIdx.x * TX, j0 = by * TY;
  const int kb = bz * g.kc, ke = kb + g.kc < g.nz ? kb + g.kc : g.nz;
  const int i = i0 + tx;
  const long P = (long)g.nx * g.ny;
  const double ir0 = 1.0 / rho0, idx = 1.0 / g.dx, idy = 1.0 / g.dy;
  const bool hxp = i + 1 < g.nx || g.bcx == 0;
  // halo cell h (threads 0 .. TY + TX - 1): column TX of rows 0..TY-1, then
  // row TY of columns 0..TX-1; wrapped when periodic, clamped (unused) at walls
  int hslot = -1;
  long hoff = 0;
  if ((int)threadIdx.x < TY + TX) {
    const int h = threadIdx.x;
    const int r = h < TY ? h : TY, c = h < TY ? TX : h - TY;
    int gi = i0 + c, gj = j0 + r;
    if (gi >= g.nx) gi = g.bcx == 0 ? 0 : g.nx - 1;
    if (gj >= g.ny) gj = g.bcy == 0 ? 0 : g.ny - 1;
    hslot = r * W + c;
    hoff = (long)gj * g.nx + gi;
  }
  long c0[RPT];
  bool hyp[RPT];
  double pc[RPT] = {}, hc[RPT] = {}, rc[RPT] = {}, fc[RPT] = {};
#pragma unroll
  for (int m = 0; m < RPT; ++m) {
    const int j = j0 + ty + 4 * m;
    c0[m] = (long)j * g.nx + i;
    hyp[m] = j + 1 < g.ny || g.bcy == 0;
    const long c = kb * P + c0[m];
    if constexpr (PHR) {
      pc[m] = p[c];
      hc[m] = ph[c];
      rc[m] = rho[c];
    }
    if constexpr (PHI) fc[m] = phi[c];
  }
  for (int k = kb; k < ke; ++k) {
    const int kp = kplus(g, k);
    const bool zph = kp >= 0 || ztop_out(g, k);
    double pp[RPT], hp[RPT], rp[RPT], fp[RPT], un[RPT], vn[RPT], wn[RPT];
    double qxv[RPT] = {}, qyv[RPT] = {}, qzv[RPT] = {};
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const long c = k * P + c0[m];
      pp[m] = hp[m] = rp[m] = fp[m] = 0.0;
      if (kp >= 0) {
        const long n = kp * P + c0[m];
        if constexpr (PHR) {
          pp[m] = p[n];
          hp[m] = ph[n];
          rp[m] = rho[n];
        }
        if constexpr (PHI) fp[m] = phi[n];
      } else if (zph) {
        pp[m] = -pc[m];
        hp[m] = -hc[m];
        rp[m] = rc[m];
        fp[m] = -fc[m];
      }
      // read once: non-temporal loads
      un[m] = __builtin_nontemporal_load(u + c);
      vn[m] = __builtin_nontemporal_load(v + c);
      wn[m] = __builtin_nontemporal_load(w + c);
      if (KIND != EPI_CORRECT && ug) {
        qxv[m] = __builtin_nontemporal_load(qx + c);
        qyv[m] = __builtin_nontemporal_load(qy + c);
        qzv[m] = __builtin_nontemporal_load(qz + c);
      }
      const int sl = (ty + 4 * m) * W + tx;
      if constexpr (PHR) {
        sm[sl] = pc[m];
        sm[AREA + sl] = hc[m];
        sm[2 * AREA + sl] = rc[m];
      }
      if constexpr (PHI) sm[3 * AREA + sl] = fc[m];
    }
    if (hslot >= 0) {
      const long n = k * P + hoff;
      if constexpr (PHR) {
        sm[hslot] = p[n];
        sm[AREA + hslot] = ph[n];
        sm[2 * AREA + hslot] = rho[n];
      }
      if constexpr (PHI) sm[3 * AREA + hslot] = phi[n];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const long c = k * P + c0[m];
      const int sl = (ty + 4 * m) * W + tx;
      double gx = 0.0, gy = 0.0, gz = 0.0;
      if constexpr (KIND == EPI_EXTEND) {
        // the gradient of phi alone (epi_face's differences)
        if (hxp) gx = (sm[3 * AREA + sl + 1] - fc[m]) * idx;
        else if (xtop_out(g)) gx = (-fc[m] - fc[m]) * idx;
        if (hyp[m]) gy = (sm[3 * AREA + sl + W] - fc[m]) * idy;
        else if (ytop_out(g)) gy = (-fc[m] - fc[m]) * idy;
        if (zph) gz = (fp[m] - fc[m]) * (1.0 / g.dzc[k]);
        const double ex = un[m] - gx, ey = vn[m] - gy, ez = wn[m] - gz;
        __builtin_nontemporal_store(ex, ue + c);
        __builtin_nontemporal_store(ey, ve + c);
        __builtin_nontemporal_store(ez, we + c);
        if (ug) {
          __builtin_nontemporal_store(ex - qxv[m], ug + c);
          __builtin_nontemporal_store(ey - qyv[m], vg + c);
          __builtin_nontemporal_store(ez - qzv[m], wg + c);
        }
      } else {
        if (hxp) {
          const int n = sl + 1;
          un[m] = epi_face(un[m], dt, ir0, sm[n], pc[m], sm[2 * AREA + n], rc[m], sm[AREA + n],
                           hc[m], PHI ? sm[3 * AREA + n] : 0.0, fc[m], idx, &gx);
        } else if (xtop_out(g)) {
          un[m] = epi_face(un[m], dt, ir0, -pc[m], pc[m], rc[m], rc[m], -hc[m], hc[m], -fc[m],
                           fc[m], idx, &gx);
        }
        if (hyp[m]) {
          const int n = sl + W;
          vn[m] = epi_face(vn[m], dt, ir0, sm[n], pc[m], sm[2 * AREA + n], rc[m], sm[AREA + n],
                           hc[m], PHI ? sm[3 * AREA + n] : 0.0, fc[m], idy, &gy);
        } else if (ytop_out(g)) {
          vn[m] = epi_face(vn[m], dt, ir0, -pc[m], pc[m], rc[m], rc[m], -hc[m], hc[m], -fc[m],
                           fc[m], idy, &gy);
        }
        if (zph)
          wn[m] = epi_face(wn[m], dt, ir0, pp[m], pc[m], rp[m], rc[m], hp[m], hc[m], fp[m], fc[m],
                           1.0 / g.dzc[k], &gz);
        if constexpr (KIND == EPI_STEP) {
          epi_store(un[m], vn[m], wn[m], gx, gy, gz, c, u, v, w, qx, qy, qz, qxv[m], qyv[m],
                    qzv[m], true, ue, ve, we, ug, vg, wg);
        } else {
          __builtin_nontemporal_store(un[m], u + c);
          __builtin_nontemporal_store(vn[m], v + c);
          __builtin_nontemporal_store(wn[m], w + c);
        }
      }
      pc[m] = pp[m];
      hc[m] = hp[m];
      rc[m] = rp[m];
      fc[m] = fp[m];
    }
    __syncthreads();  // the tile is rewritten for the next plane
  }
}

// ---------------------------------------------------------------------------
// Interface terms from the volume fraction C and the mass flux mdot (section
// 3.2: the regularised delta |grad C| by Youngs' finite differences; section
// 3.6: the Stefan source and the interface-velocity jump):
//   s = mdot (1/rho2 - 1/rho1) |grad C|             at cell centres,
//   a = (mdot / rho_e) n,  n = -grad C / |grad C|  (0 where grad C = 0):
//       the unit normal pointing into phase 2, as the Rankine-Hugoniot jump
//       condition of section 2 orients it (C is 1 in phase 1, so grad C
//       points into phase 1); rho_e is the density of the phase whose
//       velocity the extension follows: rho1, or rho2 for boiling, appendix A,
//   q on face i+1/2 = (a_i + a_{i+1}) / 2, 0 on a non-periodic boundary face.
// grad C at a centre is the mean of the gradients at its eight corners, each
// from the eight cells around the corner (ghost cells: periodic copies, or
// mirrored values at walls and outflow ends); per component that is the
// central difference weighted (1, 2, 1) / 4 in each transverse direction, in z
// the mean of the two one-sided differences over the centre distances.  The
// weights factor; differences are taken first (so a gradient at the rounding
// level of C, where C saturates at 0 or 1, stays exact):
//   dx[j][i] = sum_c w_c (C[k+c][j][i+1] - C[k+c][j][i-1]),   gx = sum_b w_b dx[j+b][i] / (32 dx),
//   dy[j][i] = sum_c w_c (C[k+c][j+1][i] - C[k+c][j-1][i]),   gy = sum_b w_b dy[j][i+b] / (32 dy),
//   zd[j][i] = (C[k+1] - C[k]) / dzc[k] + (C[k] - C[k-1]) / dzc[k-1],
//                                            gz = sum_{b,c} w_b w_c zd[j+c][i+b] / 32.
// A block owns a TX x TY tile (TX = the largest power of two dividing nx, at
// most 64, or a narrower width set by the plan; TY = 512 / TX; one cell per
// thread) and marches through g.kc planes: C of planes k-1 .. k+2 with a
// (-1, +2) x / y halo sits in a ring of four LDS planes (loads run two planes
// ahead of the computation, through registers), dx, dy and zd of the current
// plane in three more, and a of the current plane on the tile plus its +x / +y
// halo in three, so each plane of C is read about once per block.
// ---------------------------------------------------------------------------
namespace {
constexpr int kIfThreads = kInterfaceThreads;  // threads of a block = cells of its tile
// largest (TX + h)(kIfThreads / TX + h) over the tile widths TX = 8 .. 64
constexpr int if_region(int h) {
  int m = 0;
  for (int tx = 8; tx <= 64; tx *= 2) {
    const int n = (tx + h) * (kIfThreads / tx + h);
    m = n > m ? n : m;
  }
  return m;
}
constexpr int kIfMaxC = if_region(3);  // C tile with its (-1, +2) halo
constexpr int kIfMaxA = if_region(1);  // a region with its +1 halo
constexpr int kIfRegs = (kIfMaxC + kIfThreads - 1) / kIfThreads;   // C-tile values per thread
constexpr int kIfARegs = (kIfMaxA + kIfThreads - 1) / kIfThreads;  // a positions per thread

// index i of a line of n cells, periodic (any i; tall tiles of narrow grids
// reach several periods beyond the end) or mirrored into [0, n)
__device__ __forceinline__ int wrap_or_clamp(int i, int n, bool periodic) {
  if (periodic) return ((i % n) + n) % n;
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}
}  // namespace

// The march above can also carry one of the step's stencils (the interface
// terms fused into the step's first and last passes):
//   IF_RHS : at each plane p, s = mdot (1/rho2 - 1/rho1) |grad C| and the
//            pressure right-hand side b with that s (k_rhs's arithmetic);
//            s and b are written, q is not formed;
//   IF_EPI : one plane behind (plane p-1 at step p, once a of plane p is
//            known), the fused step epilogue with q = the face means of a
//            (k_step_epilogue's arithmetic); s and q are not written.
// The neighbours of a cell in the other fields are read through the caches.
enum : int { IF_TERMS = 0, IF_RHS = 1, IF_EPI = 2 };

// b at cell c = k P + j nx + i of plane k (k_rhs's arithmetic, term for term)
__device__ __forceinline__ double rhs_at(const GridArgs& g, const IfStepArgs& a, int i, int j,
                                         int k, double sv) {
  const long P = (long)g.nx * g.ny;
  const long c = k * P + (long)j * g.nx + i;
  const double ir0 = 1.0 / a.rho0, idx = 1.0 / g.dx, idy = 1.0 / g.dy, r0dt = a.rho0 / a.dt;
  const bool hxp = i + 1 < g.nx || g.bcx == 0, hxm = i > 0 || g.bcx == 0;
  const bool hyp = j + 1 < g.ny || g.bcy == 0, hym = j > 0 || g.bcy == 0;
  const long xp = i + 1 < g.nx ? 1 : -(long)(g.nx - 1), xm = i > 0 ? -1 : (long)(g.nx - 1);
  const long yp = j + 1 < g.ny ? (long)g.nx : -(long)(g.ny - 1) * g.nx;
  const long ym = j > 0 ? -(long)g.nx : (long)(g.ny - 1) * g.nx;
  const int kp = kplus(g, k), km = kminus(g, k);
  const bool zph = kp >= 0 || ztop_out(g, k);
  const double phc = a.ph[c], rhc = a.rho[c];
  double php = 0.0, rhp = 0.0;
  if (kp >= 0) {
    php = a.ph[kp * P + (c - k * P)];
    rhp = a.rho[kp * P + (c - k * P)];
  } else if (zph) {
    php = -phc;
    rhp = rhc;
  }
  double phm = 0.0, rhm = 0.0, wm = 0.0;
  if (km >= 0) {
    const long n = km * P + (c - k * P);
    phm = a.ph[n];
    rhm = a.rho[n];
    wm = a.w[n];
  }
  const RhsNbr nxp = hxp ? RhsNbr{a.ph[c + xp], a.rho[c + xp], true}
                         : RhsNbr{-phc, rhc, xtop_out(g)};
  const RhsNbr nxm{hxm ? a.ph[c + xm] : 0.0, hxm ? a.rho[c + xm] : 0.0, hxm};
  const RhsNbr nyp = hyp ? RhsNbr{a.ph[c + yp], a.rho[c + yp], true}
                         : RhsNbr{-phc, rhc, ytop_out(g)};
  const RhsNbr nym{hym ? a.ph[c + ym] : 0.0, hym ? a.rho[c + ym] : 0.0, hym};
  const RhsNbr nzp{php, rhp, zph}, nzm{phm, rhm, km >= 0};
  const double um = hxm ? a.u[c + xm] : 0.0;
  const double vm = hym ? a.v[c + ym] : 0.0;
  return rhs_cell(a.rho0, ir0, idx, idy, r0dt, phc, rhc, nxp, nxm, nyp, nym, nzp,
                  zph ? 1.0 / g.dzc[k] : 1.0, nzm, km >= 0 ? 1.0 / g.dzc[km] : 1.0,
                  1.0 / g.dzf[k], a.u[c], um, a.v[c], vm, a.w[c], wm, sv);
}

// the fused epilogue at cell (i, j, k) with the face values q of its "+"
// faces given (k_step_epilogue's arithmetic, term for term)
__device__ __forceinline__ void epi_at(const GridArgs& g, const IfStepArgs& a, int i, int j, int k,
                                       double qxv, double qyv, double qzv) {
  const long P = (long)g.nx * g.ny;
  const long c0 = (long)j * g.nx + i, c = k * P + c0;
  const double ir0 = 1.0 / a.rho0, idx = 1.0 / g.dx, idy = 1.0 / g.dy, dt = a.dt;
  const bool hxp = i + 1 < g.nx || g.bcx == 0, hyp = j + 1 < g.ny || g.bcy == 0;
  const long xp = i + 1 < g.nx ? 1 : -(long)(g.nx - 1);
  const long yp = j + 1 < g.ny ? (long)g.nx : -(long)(g.ny - 1) * g.nx;
  const int kp = kplus(g, k);
  const double pc = a.p[c], hc = a.ph[c], rc = a.rho[c], fc = a.phi[c];
  double un = a.uo[c], vn = a.vo[c], wn = a.wo[c];
  double gx = 0.0, gy = 0.0, gz = 0.0;
  if (hxp) {
    const long n = c + xp;
    un = epi_face(un, dt, ir0, a.p[n], pc, a.rho[n], rc, a.ph[n], hc, a.phi[n], fc, idx, &gx);
  } else if (xtop_out(g)) {
    un = epi_face(un, dt, ir0, -pc, pc, rc, rc, -hc, hc, -fc, fc, idx, &gx);
  }
  if (hyp) {
    const long n = c + yp;
    vn = epi_face(vn, dt, ir0, a.p[n], pc, a.rho[n], rc, a.ph[n], hc, a.phi[n], fc, idy, &gy);
  } else if (ytop_out(g)) {
    vn = epi_face(vn, dt, ir0, -pc, pc, rc, rc, -hc, hc, -fc, fc, idy, &gy);
  }
  double pp = 0.0, hp = 0.0, rp = 0.0, fp = 0.0;
  const bool zph = kp >= 0 || ztop_out(g, k);
  if (kp >= 0) {
    const long n = kp * P + c0;
    pp = a.p[n];
    hp = a.ph[n];
    rp = a.rho[n];
    fp = a.phi[n];
  } else if (zph) {
    pp = -pc;
    hp = -hc;
    rp = rc;
    fp = -fc;
  }
  if (zph) wn = epi_face(wn, dt, ir0, pp, pc, rp, rc, hp, hc, fp, fc, 1.0 / g.dzc[k], &gz);
  epi_store(un, vn, wn, gx, gy, gz, c, a.uo, a.vo, a.wo, nullptr, nullptr, nullptr, qxv, qyv, qzv,
            true, a.ue, a.ve, a.we, a.ug, a.vg, a.wg);
}

template <bool FULL, int MODE>
__global__ __launch_bounds__(kIfThreads) void k_interface(
    const GridArgs g, const double* __restrict__ C, const double* __restrict__ mdot,
    const double* __restrict__ dzc, double rho1, double rho2, double rho_e, double* __restrict__ s,
    double* __restrict__ qx, double* __restrict__ qy, double* __restrict__ qz,
    const IfStepArgs sa_args) {
  __shared__ double cs[4][kIfMaxC];
  __shared__ double sdx[kIfMaxC], sdy[kIfMaxC], zd[kIfMaxC];
  __shared__ double sax[kIfMaxA], say[kIfMaxA], saz[kIfMaxA], ssrc[kIfMaxA];
  const int tx = tile_w<64>(g);
  const int ty = kIfThreads / tx;
  const int cw = tx + 3, ch = ty + 3, aw = tx + 1, ah = ty + 1;
  const int i0 = blockIdx.x * tx, j0 = blockIdx.y * ty;
  const int kb = blockIdx.z * g.kc, ke = kb + g.kc < g.nz ? kb + g.kc : g.nz;
  const bool px = g.bcx == 0, py = g.bcy == 0, pz = g.bcz == 0;
  const long P = (long)g.nx * g.ny;
  const int li = threadIdx.x % tx, lj = threadIdx.x / tx;
  const int i = i0 + li, j = j0 + lj;
  // a cell of the domain (FULL: the tiles cover y exactly; else tall tiles of
  // narrow grids reach beyond ny)
  const bool own = FULL || j < g.ny;
  const double src_f = 1.0 / rho2 - 1.0 / rho1, a_f = -1.0 / rho_e;  // n = -grad C / |grad C|
  const double fx = 1.0 / (32.0 * g.dx), fy = 1.0 / (32.0 * g.dy);

  // This thread's C-tile elements e = threadIdx.x + kIfThreads r and a positions,
  // fixed for the march: in-plane offsets (a thread with fewer elements than
  // registers repeats its last valid one, so that every load is issued
  // unconditionally and the waits for them stay exact), which differences an
  // element carries, the centre of an a position in the C tile and whether
  // it is a cell of the block.
  long coff[kIfRegs], moff[kIfARegs];
  bool cin[kIfRegs], cdx[kIfRegs], cdy[kIfRegs], ain[kIfARegs];
  int ao[kIfARegs];
#pragma unroll
  for (int r = 0; r < kIfRegs; ++r) {
    const int e0 = threadIdx.x + kIfThreads * r, e = min(e0, cw * ch - 1);
    const int ei = e % cw, ej = e / cw;
    coff[r] = (long)wrap_or_clamp(j0 - 1 + ej, g.ny, py) * g.nx + wrap_or_clamp(i0 - 1 + ei, g.nx, px);
    cin[r] = e0 < cw * ch;
    cdx[r] = ei >= 1 && ei <= cw - 2;
    cdy[r] = ej >= 1 && ej <= ch - 2;
  }
#pragma unroll
  for (int r = 0; r < kIfARegs; ++r) {
    const int e0 = threadIdx.x + kIfThreads * r, e = min(e0, aw * ah - 1);
    const int ai = e % aw, aj = e / aw;
    moff[r] = (long)wrap_or_clamp(j0 + aj, g.ny, py) * g.nx + wrap_or_clamp(i0 + ai, g.nx, px);
    ain[r] = e0 < aw * ah;
    ao[r] = (aj + 1) * cw + (ai + 1);
  }
  // plane of index kk in [-1, nz + 1]: wrapped (periodic z, nz >= 3) or clamped
  auto plane = [&](int kk) {
    if (pz) return kk < 0 ? kk + g.nz : (kk >= g.nz ? kk - g.nz : kk);
    return kk < 0 ? 0 : (kk >= g.nz ? g.nz - 1 : kk);
  };
  auto fetch = [&](int kk, double* v) {
    const long base = (long)plane(kk) * P;
#pragma unroll
    for (int r = 0; r < kIfRegs; ++r) v[r] = C[base + coff[r]];
  };
  auto put = [&](int kk, const double* v) {
#pragma unroll
    for (int r = 0; r < kIfRegs; ++r)
      if (cin[r]) cs[kk & 3][threadIdx.x + kIfThreads * r] = v[r];
  };
  auto fetch_m = [&](int kk, double* md) {
    const long base = (long)plane(kk) * P;
#pragma unroll
    for (int r = 0; r < kIfARegs; ++r) md[r] = mdot[base + moff[r]];
  };
  // the z-weighted x and y differences and the z differences of plane kk
  // over the C tile (dx where i-1 and i+1 are in the tile, dy where j-1 and
  // j+1 are)
  auto z_sums = [&](int kk) {
    const int m = plane(kk);
    const double ihi = 1.0 / (m + 1 < g.nz ? dzc[m] : (pz ? dzc[g.nz - 1] : 1.0));
    const double ilo = 1.0 / (m > 0 ? dzc[m - 1] : (pz ? dzc[g.nz - 1] : 1.0));
    const double* cm = cs[(kk - 1) & 3];
    const double* c0 = cs[kk & 3];
    const double* cp = cs[(kk + 1) & 3];
#pragma unroll
    for (int r = 0; r < kIfRegs; ++r) {
      if (!cin[r]) break;
      const int e = threadIdx.x + kIfThreads * r;
      const double a = cm[e], b = c0[e], c = cp[e];
      zd[e] = (c - b) * ihi + (b - a) * ilo;
      if (cdx[r])
        sdx[e] = (cm[e + 1] - cm[e - 1]) + 2.0 * (c0[e + 1] - c0[e - 1]) + (cp[e + 1] - cp[e - 1]);
      if (cdy[r])
        sdy[e] = (cm[e + cw] - cm[e - cw]) + 2.0 * (c0[e + cw] - c0[e - cw]) +
                 (cp[e + cw] - cp[e - cw]);
    }
  };
  // gradient of C at a position of the a region (centre o of the C tile)
  auto grad_at = [&](int o, double& gx, double& gy, double& gz) {
    gx = (sdx[o - cw] + 2.0 * sdx[o] + sdx[o + cw]) * fx;
    gy = (sdy[o - 1] + 2.0 * sdy[o] + sdy[o + 1]) * fy;
    const double r0 = zd[o - cw - 1] + 2.0 * zd[o - cw] + zd[o - cw + 1];
    const double r1 = zd[o - 1] + 2.0 * zd[o] + zd[o + 1];
    const double r2 = zd[o + cw - 1] + 2.0 * zd[o + cw] + zd[o + cw + 1];
    gz = (r0 + 2.0 * r1 + r2) * (1.0 / 32.0);
  };
  // a of plane kk on the tile and its +x / +y halo into sax / say / saz, and
  // the source s into ssrc (mdot of this thread's positions in md)
  auto make_a = [&](const double* md) {
#pragma unroll
    for (int r = 0; r < kIfARegs; ++r) {
      if (!ain[r]) break;
      const int e = threadIdx.x + kIfThreads * r;
      double gx, gy, gz;
      grad_at(ao[r], gx, gy, gz);
      const double mag = sqrt(gx * gx + gy * gy + gz * gz);
      const double sc = mag > 0.0 ? md[r] * a_f / mag : 0.0;
      sax[e] = sc * gx;
      say[e] = sc * gy;
      saz[e] = sc * gz;
      ssrc[e] = md[r] * src_f * mag;
    }
  };

  // C of planes kb-1 .. kb+2 in the ring, then the march.  Step p computes a
  // and s of plane p and writes s, q_x, q_y of plane p (not on the last step,
  // p = ke) and q_z of plane p-1 (not on the first, p = kb; a_z of p-1 kept in
  // a register).  Loads run two steps ahead: at the end of step p the ring
  // takes plane p+3 (into the slot of plane p-1, last read by z_sums(p)) from
  // a register set, which then receives plane p+5; mdot of plane p+2 goes
  // into the set make_a(p) has just consumed.  Steps alternate between two
  // register sets (sa / sb for C, ma / mb for mdot), so no register is copied
  // while its load is in flight.  Every load is issued on every step (plane
  // indices beyond the block's range are clamped to it: a few planes are
  // read twice at the end of the march) and, with FULL tiles, every store of
  // an interior step too, so the compiler counts the outstanding memory
  // operations exactly and waits only for the loads it needs.  s and q are
  // stored non-temporally (read only by later kernels; measured at 256^3:
  // 207 -> 183 us).
  double sa[kIfRegs] = {}, sb[kIfRegs] = {}, ma[kIfARegs] = {}, mb[kIfARegs] = {};
  for (int kk = kb - 1; kk <= kb + 2; ++kk) {
    fetch(kk, sa);
    put(kk, sa);
  }
  fetch(min(kb + 3, ke + 1), sa);
  fetch(min(kb + 4, ke + 1), sb);
  fetch_m(kb, ma);
  fetch_m(kb + 1, mb);
  double az_prev = 0.0, qx_prev = 0.0, qy_prev = 0.0;
  const int ea = lj * aw + li;  // this thread's cell in the a region
  auto step = [&](int p, double* sr, double* mr, auto first_c, auto last_c) {
    constexpr bool first = decltype(first_c)::value, last = decltype(last_c)::value;
    __syncthreads();  // the ring holds planes p-1 .. p+1; the a planes are free
    z_sums(p);
    __syncthreads();
    make_a(mr);
    fetch_m(min(p + 2, ke), mr);
    __syncthreads();
    const double az = saz[ea];
    if (own) {
      const long c = p * P + (long)j * g.nx + i;
      const double qxc = (i + 1 < g.nx || px) ? 0.5 * (sax[ea] + sax[ea + 1]) : 0.0;
      const double qyc = (j + 1 < g.ny || py) ? 0.5 * (say[ea] + say[ea + aw]) : 0.0;
      if constexpr (MODE == IF_TERMS) {
        if constexpr (!last) {
          __builtin_nontemporal_store(ssrc[ea], s + c);
          __builtin_nontemporal_store(qxc, qx + c);
          __builtin_nontemporal_store(qyc, qy + c);
        }
        if constexpr (!first)
          __builtin_nontemporal_store((p < g.nz || pz) ? 0.5 * (az_prev + az) : 0.0, qz + c - P);
      } else if constexpr (MODE == IF_RHS) {
        if constexpr (!last) {
          const double sv = ssrc[ea];
          __builtin_nontemporal_store(sv, s + c);
          __builtin_nontemporal_store(rhs_at(g, sa_args, i, j, p, sv), sa_args.b + c);
        }
      } else {
        if constexpr (!first)
          epi_at(g, sa_args, i, j, p - 1, qx_prev, qy_prev,
                 (p < g.nz || pz) ? 0.5 * (az_prev + az) : 0.0);
      }
      qx_prev = qxc;
      qy_prev = qyc;
    }
    az_prev = az;
    put(p + 3, sr);  // beyond ke + 1: a clamped plane no step reads
    fetch(min(p + 5, ke + 1), sr);
  };
  using F = std::false_type;
  using T = std::true_type;
  // kc >= 1, so the march has at least the steps kb (first) and ke (last);
  // step q uses the sets a when q - kb is even
  step(kb, sa, ma, T{}, F{});
  int p = kb + 1;
  for (; p + 1 < ke; p += 2) {
    step(p, sb, mb, F{}, F{});
    step(p + 1, sa, ma, F{}, F{});
  }
  if (p < ke) {
    step(p, sb, mb, F{}, F{});
    step(ke, sa, ma, F{}, T{});
  } else {
    step(ke, sb, mb, F{}, T{});
  }
}

template <int MODE>
static hipError_t launch_interface_mode(const GridArgs& g, const double* C, const double* mdot,
                                        double rho1, double rho2, double rho_e, double* s,
                                        double* qx, double* qy, double* qz, const IfStepArgs& a,
                                        hipStream_t st) {
  const int tx = tile_w<64>(g), ty = kIfThreads / tx;
  if (tx < 8 || g.nx % tx || g.kc < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(g.nx / tx), (unsigned)((g.ny + ty - 1) / ty),
                  (unsigned)((g.nz + g.kc - 1) / g.kc));
  auto kern = g.ny % ty == 0 ? &k_interface<true, MODE> : &k_interface<false, MODE>;
  hipLaunchKernelGGL(kern, grid, dim3(kIfThreads), 0, st, g, C, mdot, g.dzc, rho1, rho2, rho_e, s,
                     qx, qy, qz, a);
  return hipGetLastError();
}

hipError_t launch_interface(const GridArgs& g, const double* C, const double* mdot, double rho1,
                            double rho2, double rho_e, double* s, double* qx, double* qy,
                            double* qz, hipStream_t st) {
  return launch_interface_mode<IF_TERMS>(g, C, mdot, rho1, rho2, rho_e, s, qx, qy, qz,
                                         IfStepArgs{}, st);
}

hipError_t launch_rhs_interface(const GridArgs& g, const double* C, const double* mdot,
                                double rho1, double rho2, double* s, const IfStepArgs& a,
                                hipStream_t st) {
  if (!a.u || !a.v || !a.w || !a.ph || !a.rho || !a.b) return hipErrorInvalidValue;
  return launch_interface_mode<IF_RHS>(g, C, mdot, rho1, rho2, rho1, s, nullptr, nullptr,
                                       nullptr, a, st);
}

hipError_t launch_epilogue_interface(const GridArgs& g, const double* C, const double* mdot,
                                     double rho_e, const IfStepArgs& a, hipStream_t st) {
  if (!a.uo || !a.vo || !a.wo || !a.p || !a.ph || !a.rho || !a.phi || !a.ug || !a.vg || !a.wg)
    return hipErrorInvalidValue;
  return launch_interface_mode<IF_EPI>(g, C, mdot, 1.0, 1.0, rho_e, nullptr, nullptr, nullptr,
                                       nullptr, a, st);
}

template <int TXMAX = 64>
static inline dim3 tile_grid(const GridArgs& g) {
  const int tx = tile_w<TXMAX>(g);
  const int ty = 256 / tx;
  return dim3((unsigned)(g.nx / tx), (unsigned)((g.ny + ty - 1) / ty),
              (unsigned)((g.nz + g.kc - 1) / g.kc));
}

int stencil_blocks(const GridArgs& g) {
  const dim3 d = tile_grid(g);
  return (int)(d.x * d.y * d.z);
}

int stencil_default_planes(int nx, int ny, int nz) {
  const int txp = nx & -nx;
  const int tx = txp < 64 ? txp : 64;
  const long tiles = (long)(nx / tx) * ((ny + 256 / tx - 1) / (256 / tx));
  long kc = (nz * tiles + 16383) / 16384;
  if (kc < 1) kc = 1;
  if (kc > nz) kc = nz;
  return (int)kc;
}

// the tiled kernel needs whole 64 x g.tiled tiles (g.tiled = 8 or 16 rows);
// g.tiled = 0 keeps the plain one
static bool rhs_tiles_fit(const GridArgs& g) {
  return (g.tiled == 8 || g.tiled == 16) && g.nx % 64 == 0 && g.ny % g.tiled == 0;
}

int rhs_blocks(const GridArgs& g) {
  if (rhs_tiles_fit(g))
    return (g.nx / 64) * (g.ny / g.tiled) * ((g.nz + g.kc - 1) / g.kc);
  return stencil_blocks(g);
}

hipError_t launch_rhs(const GridArgs& g, const double* u, const double* v, const double* w,
                      const double* phat, const double* rho, double rho0, const double* src,
                      double dt, double* b, hipStream_t st) {
  if (rhs_tiles_fit(g)) {
    const dim3 grid((unsigned)(g.nx / 64), (unsigned)(g.ny / g.tiled),
                    (unsigned)((g.nz + g.kc - 1) / g.kc));
    if (g.tiled == 16)
      hipLaunchKernelGGL(k_rhs_tiled<16>, grid, dim3(256), 0, st, g, u, v, w, phat, rho, rho0,
                         src, dt, g.dzf, g.dzc, b);
    else
      hipLaunchKernelGGL(k_rhs_tiled<8>, grid, dim3(256), 0, st, g, u, v, w, phat, rho, rho0, src,
                         dt, g.dzf, g.dzc, b);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_rhs, tile_grid(g), dim3(256), 0, st, g, u, v, w, phat, rho, rho0, src, dt,
                     b);
  return hipGetLastError();
}

// the streaming stencils (correction, extension, step epilogue) take the
// planes per block from g.kc (the plan passes its own count for them, one
// plane by default: more independent loads in flight than a march)
// LDS-staged 64 x g.tiled tiles where they fit (nx % 64 == 0, ny % g.tiled
// == 0), as the fused epilogue
static bool epi_tiles_fit(const GridArgs& g) {
  return (g.tiled == 8 || g.tiled == 16) && g.nx % 64 == 0 && g.ny % g.tiled == 0;
}

static dim3 epi_tile_grid(const GridArgs& g) {
  return dim3((unsigned)(g.nx / 64), (unsigned)(g.ny / g.tiled),
              (unsigned)((g.nz + g.kc - 1) / g.kc));
}

hipError_t launch_correct(const GridArgs& g, double* u, double* v, double* w, const double* p,
                          const double* phat, const double* rho, double rho0, double dt,
                          hipStream_t st) {
  if (epi_tiles_fit(g)) {
    auto kern = g.tiled == 16 ? &k_step_epilogue_tiled<16, EPI_CORRECT>
                              : &k_step_epilogue_tiled<8, EPI_CORRECT>;
    hipLaunchKernelGGL(kern, epi_tile_grid(g), dim3(256), 0, st, g, u, v, w, p, phat, rho, rho0,
                       dt, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                       nullptr, nullptr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_correct, tile_grid<256>(g), dim3(256), 0, st, g, u, v, w, p, phat, rho,
                     rho0, dt);
  return hipGetLastError();
}

hipError_t launch_extend(const GridArgs& g, const double* u, const double* v, const double* w,
                         const double* phi, const double* qx, const double* qy, const double* qz,
                         double* ue, double* ve, double* we, double* ug, double* vg, double* wg,
                         hipStream_t st) {
  if (epi_tiles_fit(g)) {
    auto kern = g.tiled == 16 ? &k_step_epilogue_tiled<16, EPI_EXTEND>
                              : &k_step_epilogue_tiled<8, EPI_EXTEND>;
    // u, v, w are read only in this kind
    hipLaunchKernelGGL(kern, epi_tile_grid(g), dim3(256), 0, st, g, const_cast<double*>(u),
                       const_cast<double*>(v), const_cast<double*>(w), nullptr, nullptr, nullptr,
                       1.0, 1.0, phi, qx, qy, qz, ue, ve, we, ug, vg, wg);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_extend, tile_grid<256>(g), dim3(256), 0, st, g, u, v, w, phi, qx, qy, qz,
                     ue, ve, we, ug, vg, wg);
  return hipGetLastError();
}

hipError_t launch_step_epilogue(const GridArgs& g, double* u, double* v, double* w, const double* p,
                                const double* phat, const double* rho, double rho0, double dt,
                                const double* phi, const double* qx, const double* qy,
                                const double* qz, double* ue, double* ve, double* we, double* ug,
                                double* vg, double* wg, hipStream_t st) {
  if (epi_tiles_fit(g)) {
    auto kern = g.tiled == 16 ? &k_step_epilogue_tiled<16, EPI_STEP>
                              : &k_step_epilogue_tiled<8, EPI_STEP>;
    hipLaunchKernelGGL(kern, epi_tile_grid(g), dim3(256), 0, st, g, u, v, w, p, phat, rho, rho0,
                       dt, phi, qx, qy, qz, ue, ve, we, ug, vg, wg);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_step_epilogue, tile_grid<256>(g), dim3(256), 0, st, g, u, v, w, p, phat,
                     rho, rho0, dt, phi, qx, qy, qz, ue, ve, we, ug, vg, wg);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// defect-correction control (mixed precision)
// ---------------------------------------------------------------------------
// block b: member b.  Reduces the member's x-pass partial sums (kNormSlots per
// block, nblk blocks) in a fixed order and updates state[4b + 0] = |e| of the
// step, [1] = error estimate, [2] = corrections applied; pmean[b] = the
// weighted mean of the new iterate, and after the first solve fmean[b] = the
// weighted mean of f.
//
// Error estimate of the last FP32 solve (of r, adding e to p): the chain
// rounds only what it stores, and the forward stores' rounding (at most u
// |r| each, u = 2^-24) is independent along z within a (kx, ky) line, so the
// solve amplifies it by at most `gain`, the RMS of 1/|lambda| over the z
// modes of the worst line; the inverse stores add about u |e|.  Estimate =
// 2u (gain |r| + |e|) / |p| with |r| the residual the step solved.
__global__ __launch_bounds__(256) void k_dc_update(const double* __restrict__ norms, long nblk,
                                                   int step, double tol, double gain,
                                                   double denom, double* __restrict__ state,
                                                   int* __restrict__ flags,
                                                   double* __restrict__ pmean,
                                                   double* __restrict__ fmean) {
  __shared__ double red[kNormSlots][256];
  const int b = blockIdx.x;
  // step 0 starts a solve: the member's flag (left by an earlier solve) is
  // cleared below; no pass has read it yet
  if (step > 0 && flags[b]) return;
  double v[kNormSlots] = {};
  for (long i = threadIdx.x; i < nblk; i += 256)
#pragma unroll
    for (int j = 0; j < kNormSlots; ++j) v[j] += norms[kNormSlots * (b * nblk + i) + j];
#pragma unroll
  for (int j = 0; j < kNormSlots; ++j) red[j][threadIdx.x] = v[j];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int j = 0; j < kNormSlots; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double en = sqrt(red[0][0]), pn = sqrt(red[1][0]);
  pmean[b] = red[2][0] / denom;
  double* s = state + 4 * b;
  if (step == 0) {
    fmean[b] = red[3][0] / denom;
    s[0] = en;
    s[1] = 1.0;
    s[2] = 0.0;
    flags[b] = 0;
    return;
  }
  const double rn = sqrt(red[3][0]);
  const double est = pn > 0.0 ? 0x1p-23 * (gain * rn + en) / pn : 0.0;
  s[0] = en;
  s[1] = est;
  s[2] = (double)step;
  if (tol > 0.0 && est <= tol) flags[b] = 1;
}

hipError_t launch_dc_update(const double* norms, long nblk, int nb, int step, double tol,
                            double gain, double denom, double* state, int* flags, double* pmean,
                            double* fmean, hipStream_t st) {
  if (nb < 1 || nb > kMaxBatch || nblk < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dc_update, dim3(nb), dim3(256), 0, st, norms, nblk, step, tol, gain, denom,
                     state, flags, pmean, fmean);
  return hipGetLastError();
}

}  // namespace vp

namespace vp {

// ---------------------------------------------------------------------------
// Faces at -1/2 of a lower outflow end (p = 0 on the face, half a cell before
// the first centre).  Their velocities live in one plane per direction
// (x: (j, k) at j + ny k; y: (i, k) at i + nx k; z: (i, j) at i + nx j); the
// face stencils above treat the lower end as a wall, and these kernels add
// what the outflow face changes, one launch per direction (a corner cell
// takes the terms of every direction in turn):
//   LF_RHS     b_c += -rho0 f / h - (rho0 / dt) u*_f / h,
//              f = (1/rho0 - 1/rho_c) G p_hat (rho on the face: the first cell's);
//   LF_CORRECT u_f <- u*_f - dt [ (1/rho0) G p + (1/rho_c - 1/rho0) G p_hat ];
//   LF_EXTEND  ue_f = u_f - G phi;
//   LF_STEP    LF_CORRECT, then ue_f from the corrected u_f;
// G q = (q_c - 0) / (h / 2) with h the first cell's width (dx, dy, dzf[0]).
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_lower_faces(
    const GridArgs g, int dir, double* __restrict__ uf, double* __restrict__ uef,
    double* __restrict__ b, const double* __restrict__ p, const double* __restrict__ ph,
    const double* __restrict__ rho, double rho0, double dt, const double* __restrict__ phi) {
#pragma clang fp contract(off)
  const long n1 = dir == 0 ? g.ny : g.nx, n2 = dir == 2 ? g.ny : g.nz;
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= n1 * n2) return;
  const long a = t % n1, c2 = t / n1;
  const long P = (long)g.nx * g.ny;
  // the first cell behind the face
  const long c = dir == 0 ? a * g.nx + c2 * P : (dir == 1 ? a + c2 * P : a + c2 * g.nx);
  const double h = dir == 0 ? g.dx : (dir == 1 ? g.dy : g.dzf[0]);
  const double ih = 1.0 / h, ir0 = 1.0 / rho0;
  if (MODE == LF_RHS) {
    const double f = (ir0 - 1.0 / rho[c]) * (2.0 * ph[c] * ih);
    b[c] = b[c] + (-rho0 * f * ih - (rho0 / dt) * uf[t] * ih);
    return;
  }
  double u = uf[t];
  if (MODE == LF_CORRECT || MODE == LF_STEP) {
    u = u - dt * (ir0 * (2.0 * p[c] * ih) + (1.0 / rho[c] - ir0) * (2.0 * ph[c] * ih));
    uf[t] = u;
  }
  if ((MODE == LF_EXTEND || MODE == LF_STEP) && uef) uef[t] = u - 2.0 * phi[c] * ih;
}

hipError_t launch_lower_faces(const GridArgs& g, int mode, int dir, double* uf, double* uef,
                              double* b, const double* p, const double* ph, const double* rho,
                              double rho0, double dt, const double* phi, hipStream_t st) {
  const long n = (dir == 0 ? (long)g.ny : (long)g.nx) * (dir == 2 ? (long)g.ny : (long)g.nz);
  const dim3 grid((unsigned)((n + 255) / 256));
  switch (mode) {
    case LF_RHS:
      hipLaunchKernelGGL(k_lower_faces<LF_RHS>, grid, dim3(256), 0, st, g, dir, uf, uef, b, p, ph,
                         rho, rho0, dt, phi);
      break;
    case LF_CORRECT:
      hipLaunchKernelGGL(k_lower_faces<LF_CORRECT>, grid, dim3(256), 0, st, g, dir, uf, uef, b, p,
                         ph, rho, rho0, dt, phi);
      break;
    case LF_EXTEND:
      hipLaunchKernelGGL(k_lower_faces<LF_EXTEND>, grid, dim3(256), 0, st, g, dir, uf, uef, b, p,
                         ph, rho, rho0, dt, phi);
      break;
    case LF_STEP:
      hipLaunchKernelGGL(k_lower_faces<LF_STEP>, grid, dim3(256), 0, st, g, dir, uf, uef, b, p, ph,
                         rho, rho0, dt, phi);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace vp
