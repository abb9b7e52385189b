// z pass of the spectral Poisson solve: one tridiagonal system per packed
// (x, y) coefficient, shifted by the eigenvalue lambda_x + lambda_y.
//
// Row k of the row-scaled z operator (second-order staggered difference on a
// possibly stretched z grid):
//     za[k] p[k-1] + (lambda - za[k] - zc[k]) p[k] + zc[k] p[k+1] = r[k]
// with za[k] = 1/(dzf[k] dzc[k-1]), zc[k] = 1/(dzf[k] dzc[k]); walls set
// za[0] = zc[nz-1] = 0, periodic z wraps both ends (a cyclic system).
//
// Partitioned solve (no per-element scratch in HBM): each line is cut into S
// segments; a lane owns one segment in registers.  Its interior rows satisfy
// x_i = alpha_i + beta_i x_first + gamma_i x_last in terms of the segment's
// end values; the end values of all segments then satisfy a tridiagonal
// system of 2S unknowns whose rows need alpha, gamma at the first interior
// row and alpha, beta at the last.  A forward elimination of the interior
// ends at the last interior row with its final values (and keeps its
// reciprocal pivots), an elimination from the bottom ends at the first
// interior row; the two are independent chains.  The S lanes of the line
// solve the reduced system by parallel cyclic reduction (ceil(log2 2S)
// strides instead of S dependent rows), and each lane rebuilds its interior
// by forward and back substitution with the kept pivots, its end values
// entering as the outer unknowns.  A lane thus holds two M-long arrays (the
// right-hand side and the pivots).  Lines run on consecutive lanes, so every
// load and store of a z-plane row is coalesced.  When every segment has
// exactly M rows and/or the z grid is uniform, the kernel is specialised at
// compile time (no per-row guards, constant coefficients).
//
// Accuracy.  B = -(A + lambda I) is an M-matrix whose rows all sum to
// ell = -lambda > 0 (walls and periodic ends alike: A annihilates constants).
// Every pivot is formed from row sums, in the manner of the Grassmann-
// Taksar-Heyman elimination: with off-diagonal magnitudes l_r, u_r and row
// sum rho_r, the pivot U_r = u_r + sigma_r with
//     sigma_r = rho_r + l_r sigma_{r-1} / U_{r-1},
// a sum of positive terms (the elimination from the bottom mirrors it, with
// the roles of l and u exchanged).  Forming the diagonal lambda - a - c instead
// rounds lambda against terms ~1/dz^2 and loses up to five digits on lines
// with small |lambda|.  The reduced rows keep the same form: their row sums
// are ell (1 + c tau_1) and ell (1 + a tau_{m-2}) with tau = B_int^-1 1, a
// fourth right-hand side of the interior elimination.
//
// A periodic line is solved as a wall line plus one unknown wrap flux
// F_w = (x[0] - x[nz-1]) / dzc_wrap: the wrap couplings become a flux dipole
// on the right-hand side (a second right-hand side of the reduced system,
// zero in every interior), and F_w follows from one scalar equation.
//
// An outflow end (p = 0 on the boundary face, half a cell beyond the end
// centre) adds 2 / dzf^2 of the end cell to the diagonal of B: its row sum
// becomes ell + 2 / dzf^2 > 0.  The end rows are always the first or last
// unknown of a segment, so only the reduced system sees the term (in its row
// sums rho, which keeps every pivot a sum of positive terms).  With an
// outflow end anywhere no line is singular; line (0, 0) of a plan whose only
// outflow ends are in z (lambda = 0) is then solved like any other line.
//
// Without outflow ends the (kx, ky) = (0, 0) line has lambda = 0 and is singular.  It is solved in
// conservation form instead of by elimination: after its right-hand side
// loses its dzf-weighted mean (compatibility), the face fluxes are the running
// sum F[k+1/2] = sum_{j<=k} dzf[j] r[j] (plus a constant fixed by
// periodicity when z is periodic), the values are the running sum
// p[k+1] = p[k] + dzc[k] F[k+1/2], and the result loses its weighted mean
// (the gauge of zero volume-weighted mean).  Both running sums are scans over
// the line's segments.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

#ifndef VP_PART
#define VP_PART 0  // built in two parts: 1 the FP64 kernels, 2 the FP32-storage ones
#endif
#define VP_IN_PART(k) (VP_PART == 0 || VP_PART == (k))

namespace vp {

// Reduced system of line l in M-matrix form,
//   -lo_r u_{r-1} + (rho_r + lo_r + up_r) u_r - up_r u_{r+1} = R_r,
// with one or two right-hand sides (R1, and R2 when `two`), solved by
// parallel cyclic reduction with every lane of the line at work: lane s owns
// rows 2s and 2s+1 and keeps them in registers (index q = 0, 1).  At stride d
// every row publishes itself scaled by 1/D, D = lo + up + rho (one reciprocal
// per row and stride):
//   pa = (lo/D, up/D),  pb = (rho/D, R1/D),  pc = R2/D,
// and then eliminates its neighbours at distance d (old lo_i, up_i on the right):
//   rho_i <- rho_i + lo_i (rho/D)_{i-d} + up_i (rho/D)_{i+d},  R likewise,
//   lo_i <- lo_i (lo/D)_{i-d},  up_i <- up_i (up/D)_{i+d},
// which keeps every row in row-sum form (D a sum of positive terms); after
// ceil(log2 nr) strides the rows decouple and R_i / rho_i is the solution,
// left in R1 (and R2 when `two`).  With NB = 2 the published values are
// double-buffered (buffers of nr * LB entries) and one barrier per stride
// suffices: a lane overwrites a buffer two strides later, after a barrier that
// every reader of it has passed; with NB = 1 a second barrier ends each stride.
// All lanes of the block call this.
template <int LB, int NB>
__device__ __forceinline__ void red_pcr(double2* pa, double2* pb, double* pc, double (&lo)[2],
                                        double (&up)[2], double (&rho)[2], double (&R1)[2],
                                        double (&R2)[2], bool two, int nr, int l, int s) {
  const int ne = nr * LB;
  int buf = 0;
  for (int d = 1; d < nr; d <<= 1) {
    double2* qa = pa + buf * ne;
    double2* qb = pb + buf * ne;
    double* qc = pc + buf * ne;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int o = (2 * s + q) * LB + l;
      const double id = rcp64(lo[q] + up[q] + rho[q]);
      qa[o] = make_double2(lo[q] * id, up[q] * id);
      qb[o] = make_double2(rho[q] * id, R1[q] * id);
      if (two) qc[o] = R2[q] * id;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int i = 2 * s + q;
      const double a = lo[q], b = up[q];
      double nl = 0.0, nu = 0.0;
      if (i - d >= 0) {
        const int m = (i - d) * LB + l;
        const double2 v = qb[m];
        nl = a * qa[m].x;
        rho[q] += a * v.x;
        R1[q] += a * v.y;
        if (two) R2[q] += a * qc[m];
      }
      if (i + d < nr) {
        const int p = (i + d) * LB + l;
        const double2 v = qb[p];
        nu = b * qa[p].y;
        rho[q] += b * v.x;
        R1[q] += b * v.y;
        if (two) R2[q] += b * qc[p];
      }
      lo[q] = nl;
      up[q] = nu;
    }
    if (NB == 2)
      buf ^= 1;
    else
      __syncthreads();  // one buffer: every read done before the next stride writes
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double ir = rcp64(rho[q]);
    R1[q] *= ir;
    if (two) R2[q] *= ir;
  }
}

// Largest block of the M-row kernel: 8-row segments pair with up to 1024 lanes
// (their two M-long register arrays leave room for four waves per SIMD).
constexpr int zsolve_max_threads(int M) { return M == 8 ? 1024 : 512; }

// US: every segment has exactly M rows.  UZ: uniform z spacing (interior
// coefficients a = c = A.hz2).  NB: buffers of the reduced system in LDS (2:
// one barrier per stride; 1 where two would not leave room for a second block).
template <typename T, int M, int LB, bool US, bool UZ, int NB>
__global__ __launch_bounds__(zsolve_max_threads(M)) void k_zsolve(T* __restrict__ x,
                                                                   const ZArgs A) {
  extern __shared__ __align__(16) double zsm[];
  const int S = A.nseg, nr = 2 * S;
  const bool per = A.periodic != 0;
  // published rows of the reduced system (red_pcr)
  double2* pa = reinterpret_cast<double2*>(zsm);
  double2* pb = pa + NB * nr * LB;
  double* pc = reinterpret_cast<double*>(pb + NB * nr * LB);  // periodic z only
  double* red = pc + (per ? NB * nr * LB : 0);  // [S][LB] partial sums (singular line)
  double* fin = red + S * LB;  // [4][LB] end values of a periodic line
  // stretched z: the row coefficients, shared by every line, staged once
  double* cza = fin + 4 * LB;
  double* czc = cza + A.nz;
  if (!UZ) {
    for (int k = threadIdx.x; k < A.nz; k += blockDim.x) {
      cza[k] = A.za[k];
      czc[k] = A.zc[k];
    }
    __syncthreads();
  }

  if (A.skip && A.skip[blockIdx.y]) return;  // member already converged (whole block)
  const int l = threadIdx.x % LB, s = threadIdx.x / LB;
  x += blockIdx.y * A.batch_stride;
  const long P = A.plane;
  const int k0 = US ? s * M : s * A.seg_base + (s < A.seg_rem ? s : A.seg_rem);
  const int m = US ? M : A.seg_base + (s < A.seg_rem ? 1 : 0);
  const int k1 = k0 + m - 1;
  auto coef_a = [&](int i) { return UZ ? A.hz2 : cza[k0 + i]; };
  auto coef_c = [&](int i) { return UZ ? A.hz2 : czc[k0 + i]; };
  // the segment of line t * LB + l, scaled (zero past the last line)
  auto load = [&](long t, double (&v)[M]) {
    const long ln = t * LB + l;
    const T* src = x + (long)k0 * P + ln;
#pragma unroll
    for (int i = 0; i < M; ++i)
      v[i] = ((US || i < m) && ln < P) ? double(src[(long)i * P]) * A.scale : 0.0;
  };

  // tiles of LB lines, walked with a stride of gridDim.x
  const long ntiles = (P + LB - 1) / LB;
  // the segment's right-hand side, and the reciprocal pivots of its interior
  double r[M], iu[M];
  long t = xcd_tile(blockIdx.x, gridDim.x);
  load(t, r);
  for (; t < ntiles; t += gridDim.x) {
  const long tn = t + gridDim.x;
  const long line = t * LB + l;
  const bool valid = line < P;
  const bool blk0 = t == 0;
  const bool sing = blk0 && l == 0 && A.singular;  // line 0: lambda_x + lambda_y == 0
  const bool gen = valid && !sing;
  double lam = 0.0;
  if (valid) lam = A.lamx[line % A.nx] + A.lamy[line / A.nx];
  const double ell = -lam;
  T* xs = x + (long)k0 * P + line;
  double rlast = 0.0;
#pragma unroll
  for (int i = 0; i < M; ++i)
    if (US ? i == M - 1 : i == m - 1) rlast = r[i];
  const double rfirst = r[0];

  // ---- singular line (block 0, lanes l == 0): segmented running sums ----
  if (blk0 && A.singular) {
    // sums over the segments of this lane's line (block-wide barriers)
    auto line_sum = [&](double v) -> double {
      red[s * LB + l] = v;
      __syncthreads();
      double t = 0.0;
      for (int s2 = 0; s2 < S; ++s2) t += red[s2 * LB + l];
      __syncthreads();
      return t;
    };
    auto line_excl = [&](double v) -> double {
      red[s * LB + l] = v;
      __syncthreads();
      double t = 0.0;
      for (int s2 = 0; s2 < s; ++s2) t += red[s2 * LB + l];
      __syncthreads();
      return t;
    };
    double acc = 0.0;
    if (sing) {
#pragma unroll
      for (int i = 0; i < M; ++i)
        if (i < m) acc += A.dzf[k0 + i] * r[i];
    }
    const double rbar = line_sum(acc) / A.dz_sum;
    if (sing && s == 0 && A.mean_out) A.mean_out[blockIdx.y] = rbar;
    // face fluxes F[k+1/2] (held in iu)
    double run = 0.0;
    if (sing) {
#pragma unroll
      for (int i = 0; i < M; ++i)
        if (i < m) {
          run += A.dzf[k0 + i] * (r[i] - rbar);
          iu[i] = run;
        }
    }
    double off = line_excl(run);
    if (sing) {
#pragma unroll
      for (int i = 0; i < M; ++i) iu[i] += off;
    }
    if (per) {
      // the constant flux that makes p periodic: sum_k dzc[k] F[k+1/2] = 0
      double a2 = 0.0;
      if (sing) {
#pragma unroll
        for (int i = 0; i < M; ++i)
          if (i < m) a2 += A.dzc[k0 + i] * iu[i];
      }
      const double c0 = -line_sum(a2) / A.dz_sum;
      if (sing) {
#pragma unroll
        for (int i = 0; i < M; ++i) iu[i] += c0;
      }
    }
    // values p[k] relative to the segment start (held in r: the data is used up)
    run = 0.0;
    if (sing) {
#pragma unroll
      for (int i = 0; i < M; ++i)
        if (i < m) {
          r[i] = run;
          run += A.dzc[k0 + i] * iu[i];
        }
    }
    off = line_excl(run);
    acc = 0.0;
    if (sing) {
#pragma unroll
      for (int i = 0; i < M; ++i)
        if (i < m) {
          r[i] += off;
          acc += A.dzf[k0 + i] * r[i];
        }
    }
    const double pm = line_sum(acc) / A.dz_sum;
    if (sing) {
#pragma unroll
      for (int i = 0; i < M; ++i)
        if (i < m) xs[(long)i * P] = T(r[i] - pm);
    }
  }

  // ---- interior rows 1..m-2 of B, x_i = alpha_i + beta_i x_first + gamma_i x_last
  //      with tau = B_int^-1 1: the reduced rows need alpha, gamma, tau at row 1
  //      and alpha, beta, tau at row m-2.  A forward elimination ends at row m-2
  //      with its final values and keeps its reciprocal pivots for the rebuild; an
  //      elimination from the bottom (its own row-sum pivots, an independent
  //      chain) ends at row 1.  The right-hand side of B is -r. ----
  double a1 = 0.0, g1 = 1.0, t1 = 0.0, aL = 0.0, bL = 1.0, tL = 0.0;
  {
    double ratio = 1.0, ya = 0.0, yb = 0.0, yt = 0.0;
    double rb = 1.0, za = 0.0, zg = 0.0, zt = 0.0;
    // one row of each elimination: forward row i (pivot kept), backward row j
    auto fwd = [&](int i) {
      const double a = coef_a(i), c = coef_c(i);
      const double sig = ell + a * ratio;
      const double iv = rcp64(c + sig);
      ratio = sig * iv;
      ya = (a * ya - r[i]) * iv;
      yb = (i == 1 ? a : a * yb) * iv;
      yt = (1.0 + a * yt) * iv;
      iu[i] = iv;
    };
    auto bwd = [&](int j, bool last) {
      const double a = coef_a(j), c = coef_c(j);
      const double sig = ell + c * rb;
      const double iv = rcp64(a + sig);
      rb = sig * iv;
      za = (c * za - r[j]) * iv;
      zg = (last ? c : c * zg) * iv;
      zt = (1.0 + c * zt) * iv;
    };
    if (US) {
      // equal segments: both chains in one loop (each coefficient used as loaded)
#pragma unroll
      for (int k = 1; k < M - 1; ++k) {
        fwd(k);
        bwd(M - 1 - k, k == 1);
      }
    } else {
#pragma unroll
      for (int i = 1; i < M - 1; ++i)
        if (i < m - 1) fwd(i);
#pragma unroll
      for (int i = M - 2; i >= 1; --i)
        if (i <= m - 2) bwd(i, i == m - 2);
    }
    if (US ? (M >= 3) : (m >= 3)) {
      a1 = za;
      g1 = zg;
      t1 = zt;
      aL = ya;
      bL = yb;
      tL = yt;
    }
  }

  // ---- reduced system: first and last unknown of every segment ----
  double rlo[2] = {0.0, 0.0}, rup[2] = {0.0, 0.0}, rrho[2] = {1.0, 1.0}, rR1[2] = {0.0, 0.0},
         rR2[2] = {0.0, 0.0};
  if (gen) {
    const double a0 = UZ ? (k0 == 0 ? 0.0 : A.hz2) : cza[k0];
    const double c0 = UZ ? A.hz2 : czc[k0];
    const double aE = UZ ? A.hz2 : cza[k1];
    const double cE = UZ ? (k1 == A.nz - 1 ? 0.0 : A.hz2) : czc[k1];
    rlo[0] = a0;
    rup[0] = c0 * g1;
    rrho[0] = ell * (1.0 + c0 * t1) + (k0 == 0 ? A.dlo : 0.0);
    rR1[0] = c0 * a1 - rfirst;
    rlo[1] = aE * bL;
    rup[1] = cE;
    rrho[1] = ell * (1.0 + aE * tL) + (k1 == A.nz - 1 ? A.dhi : 0.0);
    rR1[1] = aE * aL - rlast;
    // periodic: unit wrap flux entering at the first cell, leaving at the last
    if (per && s == 0) rR2[0] = -1.0 / A.dzf[0];
    if (per && s == S - 1) rR2[1] = 1.0 / A.dzf[A.nz - 1];
  }
  red_pcr<LB, NB>(pa, pb, pc, rlo, rup, rrho, rR1, rR2, per, nr, l, s);
  if (per) {
    // the end values of every line, for the wrap flux
    if (s == 0) {
      fin[l] = rR1[0];
      fin[LB + l] = rR2[0];
    }
    if (s == S - 1) {
      fin[2 * LB + l] = rR1[1];
      fin[3 * LB + l] = rR2[1];
    }
    __syncthreads();
  }

  if (gen) {
    double Ft = rR1[0], Et = rR1[1];
    if (per) {
      const double xr0 = fin[l], xrn = fin[2 * LB + l];
      const double xd0 = fin[LB + l], xdn = fin[3 * LB + l];
      const double fw = (xr0 - xrn) / (A.dzc_wrap - (xd0 - xdn));
      Ft += fw * rR2[0];
      Et += fw * rR2[1];
    }
    // interior: forward and back substitution with the stored pivots, the end
    // values entering as x_0 = Ft and x_{m-1} = Et
    double y = Ft;
#pragma unroll
    for (int i = 1; i < M - 1; ++i) {
      if (US || i < m - 1) {
        y = (coef_a(i) * y - r[i]) * iu[i];
        r[i] = y;
      }
    }
    double xn = Et;
#pragma unroll
    for (int i = M - 2; i >= 1; --i) {
      if (US || i <= m - 2) {
        xn = r[i] + coef_c(i) * iu[i] * xn;
        r[i] = xn;
      }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
      if (US || i < m) {
        double v = r[i];
        if (i == 0)
          v = Ft;
        else if ((US && i == M - 1) || (!US && i == m - 1))
          v = Et;
        xs[(long)i * P] = T(v);
      }
    }
  }
  if (tn < ntiles) load(tn, r);
  // the next tile reuses the LDS of this one (the reduced system's buffers,
  // fin): every lane has finished reading them
  if (tn < ntiles) __syncthreads();
  }  // tiles
}

// nz == 1: every line is a single unknown, x = r / (lambda - dlo - dhi)
// (0 on the singular (0,0) line)
template <typename T>
__global__ __launch_bounds__(256) void k_z1(T* __restrict__ x, const ZArgs A) {
  const long line = (long)blockIdx.x * 256 + threadIdx.x;
  if (line >= A.plane || (A.skip && A.skip[blockIdx.y])) return;
  x += blockIdx.y * A.batch_stride;
  const double r = double(x[line]) * A.scale;
  if (line == 0 && A.singular) {
    if (A.mean_out) A.mean_out[blockIdx.y] = r;
    x[0] = T(0);
  } else {
    const double lam = A.lamx[line % A.nx] + A.lamy[line / A.nx] - (A.dlo + A.dhi);
    x[line] = T(r / lam);
  }
}

// LDS of one block: the reduced system's published rows (NB buffers of nr * LB
// entries: two double2 arrays, one double array when z is periodic), the
// singular line's partial sums, a periodic line's end values, and the row
// coefficients of a stretched grid.
static size_t zsolve_lds(const ZArgs& a, int lb, int nbuf, bool uz) {
  const size_t ne = (size_t)2 * a.nseg * lb;
  return sizeof(double) * ((4 + (a.periodic ? 1 : 0)) * (size_t)nbuf * ne +
                           (size_t)a.nseg * lb + 4 * (size_t)lb + (uz ? 0 : 2 * (size_t)a.nz));
}

template <typename T, int M, int LB, bool US, bool UZ>
static hipError_t launch_z_shape(T* data, const ZArgs& a, int nb, hipStream_t st) {
  const int threads = LB * a.nseg;
  if (threads > zsolve_max_threads(M)) return hipErrorInvalidValue;
  // two buffers where they leave room for as many blocks as the lanes allow
  // (four waves per SIMD, 160 KB of LDS per CU)
  const int blocks_cu = threads >= 1024 ? 1 : 1024 / threads;
  const bool two = zsolve_lds(a, LB, 2, UZ) * blocks_cu <= 163840;
  const size_t shm = zsolve_lds(a, LB, two ? 2 : 1, UZ);
  const dim3 grid((unsigned)((a.plane + LB - 1) / LB), (unsigned)nb);
  auto kern = two ? &k_zsolve<T, M, LB, US, UZ, 2> : &k_zsolve<T, M, LB, US, UZ, 1>;
  if (shm > 163840) return hipErrorInvalidValue;
  if (shm > 65536 && allow_large_lds(kern) != hipSuccess) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kern, grid, dim3((unsigned)threads), shm, st, data, a);
  return hipGetLastError();
}

template <typename T, int M, int LB>
static hipError_t launch_z_lb(T* data, const ZArgs& a, int nb, hipStream_t st) {
  const bool us = a.seg_rem == 0 && a.seg_base == M;
  if (us)
    return a.uniform_z ? launch_z_shape<T, M, LB, true, true>(data, a, nb, st)
                       : launch_z_shape<T, M, LB, true, false>(data, a, nb, st);
  return a.uniform_z ? launch_z_shape<T, M, LB, false, true>(data, a, nb, st)
                     : launch_z_shape<T, M, LB, false, false>(data, a, nb, st);
}

template <typename T, int M>
static hipError_t launch_z_m(T* data, const ZArgs& a, int nb, hipStream_t st) {
  // LB lines x S segments per block; a.lines picks LB, halved until the block
  // fits
  int lb = a.lines;
  while (lb > 8 && lb * a.nseg > zsolve_max_threads(M)) lb /= 2;
  if (lb * a.nseg > zsolve_max_threads(M)) return hipErrorInvalidValue;
  if (lb >= 32) return launch_z_lb<T, M, 32>(data, a, nb, st);
  if (lb == 16) return launch_z_lb<T, M, 16>(data, a, nb, st);
  return launch_z_lb<T, M, 8>(data, a, nb, st);
}

template <typename T>
static hipError_t launch_z(T* data, const ZArgs& a, int nb, hipStream_t st) {
  if (nb < 1 || nb > kMaxBatch) return hipErrorInvalidValue;
  if (a.nz == 1) {
    const dim3 grid((unsigned)((a.plane + 255) / 256), (unsigned)nb);
    hipLaunchKernelGGL((k_z1<T>), grid, dim3(256), 0, st, data, a);
    return hipGetLastError();
  }
  if (a.seg_base > a.seg || (a.seg_base == a.seg && a.seg_rem > 0)) return hipErrorInvalidValue;
  switch (a.seg) {
    case 8: return launch_z_m<T, 8>(data, a, nb, st);
    case 16: return launch_z_m<T, 16>(data, a, nb, st);
    default: return hipErrorInvalidValue;
  }
}

#if VP_IN_PART(1)
hipError_t launch_zsolve_f64(double* data, const ZArgs& a, int nb, hipStream_t st) {
  return launch_z<double>(data, a, nb, st);
}
#endif
#if VP_IN_PART(2)
hipError_t launch_zsolve_f32(float* data, const ZArgs& a, int nb, hipStream_t st) {
  return launch_z<float>(data, a, nb, st);
}
#endif

}  // namespace vp
