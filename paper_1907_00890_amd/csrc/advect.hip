// VoF advection of section 3.1: the volume fraction C carried by the
// interface velocity u_Gamma of section 3.6 (eq. cadv) with directional
// splitting, x then y then z (eq. fluxes), each sweep implicit in its own
// result through the divergence of its velocity component, and the final
// correction with the implicit volume-deflation term (eq. final_corr_2; the
// original correction eq. final_corr_1 on request).
//
// Flux: the MTHINC method the paper cites (Ii et al., J. Comput. Phys. 231,
// 2012), linear reconstruction.  In a cell with local coordinates
// X in [-1/2, 1/2]^3 the indicator is H = 1/2 (1 + tanh(beta (m.X + d))),
// m the unit normal of the Youngs gradient in cell coordinates
// (dx g_x, dy g_y, dz_k g_z), d fixed by the cell's volume (the integral of H
// over the cell is C).  Integrals of H over a box of the cell are exact along
// the dominant axis of m (the first of x, y, z within a factor 1 - 1e-9 of
// the largest component) and 2-point Gauss-Legendre in the other two.  The
// flux through a face of velocity V is sign(V) h times the integral over the
// part of the upwind cell (width h along the sweep) that the face sweeps in
// dt, the last xi = |V| dt / h of it (clamped to 1).  Cells with C within
// 1e-8 of 0 or 1, or a change of C across the cell below 1e-12, are uniform
// (H = C); ghost cells beyond a non-periodic end are uniform with the end
// cell's C.  The face at -1/2 of a lower outflow end takes its velocity
// from a plane (x: (j, k) at j + ny k; y: (i, k) at i + nx k; z: (i, j) at
// i + nx j).
//
// Launch shape: one thread per cell, 256 per block.  Every face flux is
// computed once and used by both cells sharing the face (LDS within the x and
// y tiles, a register carried from plane to plane in the z march; the faces
// on a tile's lower edge are computed by both tiles with the same function of
// the same data), so the fluxes telescope exactly and the scheme's volume
// balance holds to the rounding of the updates alone.  The reconstruction
// runs only where the upwind cell is an interface cell (a band); elsewhere a
// face costs its velocity and the upwind C.  In the x sweep the band's faces
// of a block are gathered into an LDS queue and computed by all its threads
// together.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace vp {

namespace {

constexpr double kBandEps = 1e-8;
constexpr double kGradMin = 1e-12;
constexpr double kAxisTol = 1e-9;
constexpr double kGauss = 0.28867513459481287;  // 1 / (2 sqrt 3): 2-point nodes on [-1/2, 1/2]

__device__ __forceinline__ int wrap_clamp(int i, int n, bool periodic) {
  if (periodic) return ((i % n) + n) % n;
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// the reconstruction of one cell
struct Rec {
  double m0, m1, m2;  // unit normal in cell coordinates (x, y, z)
  double d;
  int a;              // dominant axis
};

__device__ __forceinline__ double comp(const Rec& r, int ax) {
  return ax == 0 ? r.m0 : (ax == 1 ? r.m1 : r.m2);
}

// Youngs gradient of C at cell (i, j, k) scaled to cell coordinates:
// (dx g_x, dy g_y, dzf_k g_z).  g is the mean of the gradients at the cell's
// eight corners, each from the eight cells around the corner; per component
// the central difference weighted (1, 2, 1) in each transverse direction,
// in z the mean of the two one-sided differences over the centre distances.
// Ghost cells: periodic copies, or the end cell's value.
__device__ void youngs_scaled(const GridArgs& g, const double* __restrict__ C, int i, int j, int k,
                              double& hx, double& hy, double& hz) {
#pragma clang fp contract(off)
  const bool px = g.bcx == 0, py = g.bcy == 0, pz = g.bcz == 0;
  int ii[3], jj[3], kk[3];
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    ii[o] = wrap_clamp(i + o - 1, g.nx, px);
    jj[o] = wrap_clamp(j + o - 1, g.ny, py);
    kk[o] = wrap_clamp(k + o - 1, g.nz, pz);
  }
  double c[3][3][3];  // [dz][dy][dx]
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int o = 0; o < 3; ++o)
        c[a][b][o] = C[(long)ii[o] + (long)g.nx * (jj[b] + (long)g.ny * kk[a])];
  const double w[3] = {1.0, 2.0, 1.0};
  // centre distances across the faces k-1/2 and k+1/2 (the difference across
  // a ghost face is zero, its distance only has to be positive)
  const double dzc_m = k > 0 ? g.dzc[k - 1] : (pz ? g.dzc[g.nz - 1] : 1.0);
  const double dzc_p = k + 1 < g.nz ? g.dzc[k] : (pz ? g.dzc[g.nz - 1] : 1.0);
  double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      sx += w[a] * w[b] * (c[a][b][2] - c[a][b][0]);
      sy += w[a] * w[b] * (c[a][2][b] - c[a][0][b]);
      sz += w[a] * w[b] * ((c[2][a][b] - c[1][a][b]) / dzc_p + (c[1][a][b] - c[0][a][b]) / dzc_m);
    }
  const double gx = sx / (32.0 * g.dx), gy = sy / (32.0 * g.dy), gz = sz / 32.0;
  hx = g.dx * gx;
  hy = g.dy * gy;
  hz = g.dzf[k] * gz;
}

// Integral of H over the box that is [s0, s1] along axis `ax` and the whole
// cell along the other two; also its first and second derivatives with
// respect to d (d tanh/dx = 1 - tanh^2).
__device__ void box_integral(const Rec& r, int ax, double s0, double s1, double beta, double& val,
                             double& dval, double& d2val) {
#pragma clang fp contract(off)
  const int a = r.a;
  const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
  const double ma = comp(r, a), m1 = comp(r, t1), m2 = comp(r, t2);
  // extent of each axis: [s0, s1] along ax, [-1/2, 1/2] otherwise
  const double a0 = ax == a ? s0 : -0.5, a1 = ax == a ? s1 : 0.5;
  const double lo1 = ax == t1 ? s0 : -0.5, hi1 = ax == t1 ? s1 : 0.5;
  const double lo2 = ax == t2 ? s0 : -0.5, hi2 = ax == t2 ? s1 : 0.5;
  const double c1 = 0.5 * (lo1 + hi1), r1 = hi1 - lo1;
  const double c2 = 0.5 * (lo2 + hi2), r2 = hi2 - lo2;
  const double inv = 1.0 / (2.0 * beta * ma);
  double tot = 0.0, dtot = 0.0, d2tot = 0.0;
#pragma unroll
  for (int p = -1; p <= 1; p += 2)
#pragma unroll
    for (int q = -1; q <= 1; q += 2) {
      const double y = c1 + (double)p * kGauss * r1;
      const double z = c2 + (double)q * kGauss * r2;
      const double A = r.d + m1 * y + m2 * z;
      const double x1 = beta * (ma * a1 + A), x0 = beta * (ma * a0 + A);
      // lncosh(x1) - lncosh(x0) = |x1| - |x0| + ln((1 + e1) / (1 + e0)) with
      // e = exp(-2|x|): one logarithm, of 1 + (e1 - e0) / (1 + e0)
      const double e1 = exp(-2.0 * fabs(x1)), e0 = exp(-2.0 * fabs(x0));
      const double dl = (fabs(x1) - fabs(x0)) + log1p((e1 - e0) / (1.0 + e0));
      const double J = 0.5 * (a1 - a0) + dl * inv;
      const double t1 = copysign((1.0 - e1) / (1.0 + e1), x1);
      const double t0 = copysign((1.0 - e0) / (1.0 + e0), x0);
      const double dJ = (t1 - t0) * (beta * inv);
      const double d2J = (t0 - t1) * (t0 + t1) * (beta * beta * inv);
      tot = tot + 0.25 * r1 * r2 * J;
      dtot = dtot + 0.25 * r1 * r2 * dJ;
      d2tot = d2tot + 0.25 * r1 * r2 * d2J;
    }
  val = tot;
  dval = dtot;
  d2val = d2tot;
}

// d with the integral of H over the cell equal to C: safeguarded Halley
// iteration (the second derivative of the volume comes with the first, from
// the same tanh values) from the one-dimensional closed form along the
// dominant axis, inside the bracket [-(2 + 25 / beta), 2 + 25 / beta]
// (bisection where a step leaves it or the Halley denominator is not
// positive).  The volume error falls cubically from the first guess (about
// 1e-2) to the rounding level of its O(10)-sized terms (a few 1e-15).  The
// solve stops after the regular step taken from a volume error below 1e-13
// or after a regular step below 1e-8 (1 + |d|): with cubic convergence that
// step's result is already at the rounding level; or when a step vanishes in
// rounding.  A step landing on a bracket end is a regular step (the end is
// the last iterate once the step is below half an ulp), not a reason to
// bisect.
__device__ double solve_d(Rec& r, double C, double beta) {
#pragma clang fp contract(off)
  const double ma = fabs(comp(r, r.a));
  const double bp = beta * ma;
  const double R = exp(bp * (2.0 * C - 1.0)), b = exp(bp);
  double d = ma * (log((R * b - 1.0) / (b - R)) / (2.0 * bp));
  const double span = 2.0 + 25.0 / beta;
  double lo = -span, hi = span;
  if (!(d > lo && d < hi)) d = 0.0;
  for (int it = 0; it < 40; ++it) {
    r.d = d;
    double f, df, d2f;
    box_integral(r, 0, -0.5, 0.5, beta, f, df, d2f);
    f = f - C;
    if (f == 0.0) break;
    if (f < 0.0) lo = d;
    else hi = d;
    const double den = 2.0 * df * df - f * d2f;
    double dn = d - 2.0 * f * df / den;
    const bool regular = df > 0.0 && den > 0.0 && dn >= lo && dn <= hi;
    if (!regular) dn = 0.5 * (lo + hi);
    if (dn == d) break;
    const double step = fabs(dn - d);
    d = dn;
    if (regular && (fabs(f) <= 1e-13 || step <= 1e-8 * (1.0 + fabs(d)))) break;
  }
  r.d = d;
  return d;
}

// index helpers of a sweep along AX
template <int AX>
__device__ __forceinline__ int extent(const GridArgs& g) {
  return AX == 0 ? g.nx : (AX == 1 ? g.ny : g.nz);
}
template <int AX>
__device__ __forceinline__ bool periodic_along(const GridArgs& g) {
  return (AX == 0 ? g.bcx : (AX == 1 ? g.bcy : g.bcz)) == 0;
}
template <int AX>
__device__ __forceinline__ double width(const GridArgs& g, int s) {
  return AX == 0 ? g.dx : (AX == 1 ? g.dy : g.dzf[s]);
}

// Flux through the face between cells f - 1 and f along AX (f = 0 .. n, the
// cells' other coordinates i, j, k), with face velocity V.
template <int AX>
__device__ double face_flux(const GridArgs& g, const double* __restrict__ C, int f, int i, int j,
                            int k, double V, double dt, double beta) {
#pragma clang fp contract(off)
  if (V == 0.0) return 0.0;
  const int n = extent<AX>(g);
  const bool per = periodic_along<AX>(g);
  const bool pos = V > 0.0;
  int up = pos ? f - 1 : f;
  const bool ghost = !per && (up < 0 || up >= n);
  up = wrap_clamp(up, n, per);
  const int ci = AX == 0 ? up : i, cj = AX == 1 ? up : j, ck = AX == 2 ? up : k;
  const double cu = C[(long)ci + (long)g.nx * (cj + (long)g.ny * ck)];
  const double h = width<AX>(g, AX == 2 ? ck : 0);
  double xi = fabs(V) * dt / h;
  xi = xi < 1.0 ? xi : 1.0;
  const double sgn = pos ? 1.0 : -1.0;
  if (ghost || !(cu > kBandEps && cu < 1.0 - kBandEps)) return sgn * h * xi * cu;
  double hx, hy, hz;
  youngs_scaled(g, C, ci, cj, ck, hx, hy, hz);
  const double mag = sqrt(hx * hx + hy * hy + hz * hz);
  if (!(mag > kGradMin)) return sgn * h * xi * cu;
  Rec r;
  r.m0 = hx / mag;
  r.m1 = hy / mag;
  r.m2 = hz / mag;
  const double a0 = fabs(r.m0), a1 = fabs(r.m1), a2 = fabs(r.m2);
  const double big = fmax(a0, fmax(a1, a2)) * (1.0 - kAxisTol);
  r.a = a0 >= big ? 0 : (a1 >= big ? 1 : 2);
  solve_d(r, cu, beta);
  double I, dI, d2I;
  if (pos) box_integral(r, AX, 0.5 - xi, 0.5, beta, I, dI, d2I);
  else box_integral(r, AX, -0.5, -0.5 + xi, beta, I, dI, d2I);
  return sgn * h * I;
}

// Whether face_flux of this face takes the reconstruction (its upwind cell is
// an interface cell and not a ghost): the same tests in the same order.
template <int AX>
__device__ __forceinline__ bool face_in_band(const GridArgs& g, const double* __restrict__ C,
                                             int f, int i, int j, int k, double V) {
  if (V == 0.0) return false;
  const int n = extent<AX>(g);
  const bool per = periodic_along<AX>(g);
  int up = V > 0.0 ? f - 1 : f;
  if (!per && (up < 0 || up >= n)) return false;
  up = wrap_clamp(up, n, per);
  const int ci = AX == 0 ? up : i, cj = AX == 1 ? up : j, ck = AX == 2 ? up : k;
  const double cu = C[(long)ci + (long)g.nx * (cj + (long)g.ny * ck)];
  return cu > kBandEps && cu < 1.0 - kBandEps;
}

// The cell update of a split step along AX from its two face fluxes:
// (C - (f_{s+1/2} - f_{s-1/2}) / h) / (1 - dt (V_{s+1/2} - V_{s-1/2}) / h);
// FINAL (AX = 2) adds the final correction of the three sweeps with C1 (the
// x sweep's result at the cell; may alias out) and the x / y face
// velocities u, v:  F = C1 du/dx + C2 dv/dy + C3 dw/dz,
//   deflation: out = (C3 - dt F) / (1 - dt (du/dx + dv/dy + dw/dz)),  else C3 - dt F.
template <int AX, bool FINAL>
__device__ __forceinline__ void update_cell(const GridArgs& g, const double* __restrict__ C,
                                            long idx, int i, int j, double h, double vlo,
                                            double vup, double flo, double fup, double* out,
                                            double dt, int deflation, const double* C1,
                                            const double* __restrict__ u,
                                            const double* __restrict__ v,
                                            const double* __restrict__ lox,
                                            const double* __restrict__ loy) {
#pragma clang fp contract(off)
  const double delta = (vup - vlo) / h;
  const double cn = (C[idx] - (fup - flo) / h) / (1.0 - dt * delta);
  if (!FINAL) {
    out[idx] = cn;
    return;
  }
  const long P = (long)g.nx * g.ny, k = idx / P;
  const double uup = u[idx];
  const double ulo = i > 0 ? u[idx - 1]
                           : (g.bcx == 0 ? u[idx + g.nx - 1] : (lox ? lox[j + (long)g.ny * k] : 0.0));
  const double wy = v[idx];
  const double wyl = j > 0 ? v[idx - g.nx]
                           : (g.bcy == 0 ? v[idx + (long)(g.ny - 1) * g.nx]
                                         : (loy ? loy[i + (long)g.nx * k] : 0.0));
  const double ddx = (uup - ulo) / g.dx, ddy = (wy - wyl) / g.dy;
  const double F = C1[idx] * ddx + C[idx] * ddy + cn * delta;
  const double r = cn - dt * F;
  out[idx] = deflation ? r / (1.0 - dt * (ddx + ddy + delta)) : r;
}

// x and y sweeps: a TX x TY tile of one plane, one thread per cell.  Each
// thread takes the flux of its cell's upper face into LDS; the first cell of
// each line along the sweep also takes its lower face; the update reads both
// faces from LDS, so every face of the tile is computed once.  Faces whose
// upwind cell needs the reconstruction are not computed by their owner: they
// go to a queue in LDS (owner, which face, velocity), and all threads of the
// block then work through the queue, so the interface cells of the tile fill
// whole wavefronts instead of idling most lanes of every wavefront that holds
// one (x sweep: 1.54 -> 1.26 ms at 256^3; the y sweep and the z march measured
// no gain, so they compute every face in its owner).  The flux of a face is the
// same function of the same data whichever thread computes it.
template <int AX>
__global__ __launch_bounds__(256) void k_adv_xy(const GridArgs g, int tx,
                                               const double* __restrict__ C,
                                               const double* __restrict__ V,
                                               const double* __restrict__ lo,
                                               double* __restrict__ out, double dt, double beta) {
#pragma clang fp contract(off)
  constexpr int kFaces = 256 + 64;  // upper faces, and at most 64 line-first lower faces
  __shared__ double fl[kFaces];
  __shared__ double qv[kFaces];  // queued faces: velocity
  __shared__ int qe[kFaces];     // queued faces: owner thread * 2 + (1: lower face)
  __shared__ int qn;
  const int ltx = __builtin_ctz(tx);
  const int ty = 256 >> ltx;
  const int n = extent<AX>(g);
  const bool per = periodic_along<AX>(g);
  const long stride = AX == 0 ? 1L : (long)g.nx;
  const int k = blockIdx.z;
  // cell, and LDS slots of its faces, of thread t: x sweep, row lj holds faces
  // i0-1/2 .. i0+tx-1/2 at lj * (tx + 1) + 0 .. tx; y sweep, face row
  // r = 0 .. ty at r * tx + li
  auto cell_of = [&](int t, int& i, int& j, int& up_slot, int& lo_slot) {
    const int li = t & (tx - 1), lj = t >> ltx;
    i = blockIdx.x * tx + li;
    j = blockIdx.y * ty + lj;
    up_slot = AX == 0 ? lj * (tx + 1) + li + 1 : (lj + 1) * tx + li;
    lo_slot = AX == 0 ? lj * (tx + 1) + li : lj * tx + li;
  };
  int i, j, up_slot, lo_slot;
  cell_of(threadIdx.x, i, j, up_slot, lo_slot);
  const bool own = j < g.ny;
  const long idx = (long)i + (long)g.nx * ((own ? j : 0) + (long)g.ny * k);
  const int s = AX == 0 ? i : j;
  const bool first = (AX == 0 ? (int)(threadIdx.x & (tx - 1)) : (int)(threadIdx.x >> ltx)) == 0;
  // the queue pays in the x sweep, whose tile rows collect a row's interface
  // faces; in the y sweep (16 x 16 tiles) it measured no gain
  constexpr bool QUEUE = AX == 0;
  if (threadIdx.x == 0) qn = 0;
  __syncthreads();
  double vup = 0.0, vlo = 0.0;
  if (own) {
    vup = V[idx];
    // the face at -1/2: wrapped, a lower outflow face (its plane), or a wall
    const long lof = AX == 0 ? j + (long)g.ny * k : i + (long)g.nx * k;
    vlo = s > 0 ? V[idx - stride]
                : (per ? V[idx + (long)(n - 1) * stride] : (lo ? lo[lof] : 0.0));
    if (QUEUE && face_in_band<AX>(g, C, s + 1, i, j, k, vup)) {
      const int q = atomicAdd(&qn, 1);
      qe[q] = 2 * (int)threadIdx.x;
      qv[q] = vup;
    } else {
      fl[up_slot] = face_flux<AX>(g, C, s + 1, i, j, k, vup, dt, beta);
    }
    if (first) {
      if (QUEUE && face_in_band<AX>(g, C, s, i, j, k, vlo)) {
        const int q = atomicAdd(&qn, 1);
        qe[q] = 2 * (int)threadIdx.x + 1;
        qv[q] = vlo;
      } else {
        fl[lo_slot] = face_flux<AX>(g, C, s, i, j, k, vlo, dt, beta);
      }
    }
  }
  __syncthreads();
  const int nq = qn;
  for (int e = threadIdx.x; e < nq; e += 256) {
    const int t = qe[e] >> 1;
    const bool lower = qe[e] & 1;
    int it, jt, us, ls;
    cell_of(t, it, jt, us, ls);
    const int st = AX == 0 ? it : jt;
    fl[lower ? ls : us] = face_flux<AX>(g, C, lower ? st : st + 1, it, jt, k, qv[e], dt, beta);
  }
  __syncthreads();
  if (!own) return;
  update_cell<AX, false>(g, C, idx, i, j, width<AX>(g, 0), vlo, vup, fl[lo_slot], fl[up_slot], out,
                         dt, 0, nullptr, nullptr, nullptr, nullptr, nullptr);
}

// z sweep with the final correction: a TX x TY tile of the x-y plane marching
// through kc planes; the flux of the upper face of plane k is carried to
// plane k+1 as its lower face, so each face is computed once (the block's
// first lower face aside).
__global__ __launch_bounds__(256) void k_adv_z(const GridArgs g, int tx, int kc,
                                              const double* __restrict__ C,
                                              const double* __restrict__ W, double* out,
                                              double dt, double beta, int deflation,
                                              const double* C1, const double* __restrict__ u,
                                              const double* __restrict__ v,
                                              const double* __restrict__ lox,
                                              const double* __restrict__ loy,
                                              const double* __restrict__ loz) {
#pragma clang fp contract(off)
  const int ltx = __builtin_ctz(tx);
  const int ty = 256 >> ltx;
  const int i = blockIdx.x * tx + (threadIdx.x & (tx - 1));
  const int j = blockIdx.y * ty + (threadIdx.x >> ltx);
  if (j >= g.ny) return;
  const int kb = blockIdx.z * kc, ke = kb + kc < g.nz ? kb + kc : g.nz;
  const bool per = g.bcz == 0;
  const long P = (long)g.nx * g.ny;
  const long col = (long)i + (long)g.nx * j;
  double vlo = kb > 0 ? W[col + (long)(kb - 1) * P]
                      : (per ? W[col + (long)(g.nz - 1) * P] : (loz ? loz[col] : 0.0));
  double flo = face_flux<2>(g, C, kb, i, j, kb, vlo, dt, beta);
  for (int k = kb; k < ke; ++k) {
    const long idx = col + (long)k * P;
    const double vup = W[idx];
    const double fup = face_flux<2>(g, C, k + 1, i, j, k, vup, dt, beta);
    update_cell<2, true>(g, C, idx, i, j, g.dzf[k], vlo, vup, flo, fup, out, dt, deflation, C1, u,
                         v, lox, loy);
    vlo = vup;
    flo = fup;
  }
}

}  // namespace

hipError_t launch_advect(const GridArgs& g, const double* C, const double* ug, const double* vg,
                         const double* wg, const double* const* lo, double dt, double beta,
                         int deflation, double* work, double* out, int sweep, hipStream_t st) {
  if (g.txp < 1 || g.nx % g.txp) return hipErrorInvalidValue;
  // x sweep: 64-wide tiles (rows of faces, one extra face per row); y sweep:
  // 16-wide tiles, 16 rows (one extra row of faces per 16); z sweep: 64 x 4
  // tiles marching 16 planes
  const int tx = sweep == 1 ? (g.txp < 16 ? g.txp : 16) : (g.txp < 64 ? g.txp : 64);
  const int ty = 256 / tx;
  const unsigned bx = (unsigned)(g.nx / tx), by = (unsigned)((g.ny + ty - 1) / ty);
  // x: C -> out (C*); y: out -> work (C**); z: work -> out (C^{n+1}), with C* read from out
  if (sweep == 0) {
    hipLaunchKernelGGL((k_adv_xy<0>), dim3(bx, by, (unsigned)g.nz), dim3(256), 0, st, g, tx, C, ug,
                       lo[0], out, dt, beta);
  } else if (sweep == 1) {
    hipLaunchKernelGGL((k_adv_xy<1>), dim3(bx, by, (unsigned)g.nz), dim3(256), 0, st, g, tx, out,
                       vg, lo[1], work, dt, beta);
  } else {
    const int kc = g.nz < 16 ? g.nz : 16;
    hipLaunchKernelGGL(k_adv_z, dim3(bx, by, (unsigned)((g.nz + kc - 1) / kc)), dim3(256), 0, st, g,
                       tx, kc, work, wg, out, dt, beta, deflation, out, ug, vg, lo[0], lo[1], lo[2]);
  }
  return hipGetLastError();
}

}  // namespace vp
