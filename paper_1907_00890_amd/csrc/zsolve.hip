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
// segments; a lane owns one segment in registers and eliminates its interior
// rows for the data and for the two couplings to the segment's end values
// (x_i = alpha_i + beta_i x_first + gamma_i x_last).  The end values of all
// segments then satisfy a tridiagonal system of 2S unknowns, which the S
// lanes of the line solve in LDS by parallel cyclic reduction (ceil(log2 2S)
// strides instead of S dependent rows); each lane finally rebuilds its
// interior.  Lines run on
// consecutive lanes, so every load and store of a z-plane row is coalesced.
// When every segment has exactly M rows and/or the z grid is uniform, the
// kernel is specialised at compile time (no per-row guards, constant
// coefficients).
//
// Accuracy.  B = -(A + lambda I) is an M-matrix whose rows all sum to
// ell = -lambda > 0 (walls and periodic ends alike: A annihilates constants).
// Every pivot is formed from row sums, in the manner of the Grassmann-
// Taksar-Heyman elimination: with off-diagonal magnitudes l_r, u_r and row
// sum rho_r, the pivot U_r = u_r + sigma_r with
//     sigma_r = rho_r + l_r sigma_{r-1} / U_{r-1},
// a sum of positive terms.  Forming the diagonal lambda - a - c instead
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

namespace vp {

// Reduced system of line l (rows r*LB + l) in M-matrix form,
//   -lo_r u_{r-1} + (rho_r + lo_r + up_r) u_r - up_r u_{r+1} = R_r,
// with one or two right-hand sides (R1, and R2 when `two`), solved by
// parallel cyclic reduction with every lane of the line at work: lane s owns
// rows 2s and 2s+1.  At stride d each row
// eliminates its neighbours at distance d,
//   a = lo_i / D_{i-d},  b = up_i / D_{i+d}   (D = lo + up + rho),
//   lo_i <- a lo_{i-d},  up_i <- b up_{i+d},  rho_i <- rho_i + a rho_{i-d} + b rho_{i+d},
//   R_i <- R_i + a R_{i-d} + b R_{i+d},
// which keeps every row in row-sum form (D a sum of positive terms); after
// ceil(log2 nr) strides the rows decouple and R_i / rho_i is the solution,
// written to R1 (and R2 when `two`).  All lanes of the block call this.
template <int LB>
__device__ __forceinline__ void red_pcr(double* lo, double* up, double* rho, double* R1,
                                        double* R2, bool two, int nr, int l, int s) {
  for (int d = 1; d < nr; d <<= 1) {
    double nlo[2], nup[2], nrh[2], n1[2], n2[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int i = 2 * s + q;
      const int o = i * LB + l;
      double rh = rho[o], a1 = R1[o], a2 = two ? R2[o] : 0.0, l2 = 0.0, u2 = 0.0;
      if (i - d >= 0) {
        const int m = (i - d) * LB + l;
        const double a = lo[o] * rcp64(lo[m] + up[m] + rho[m]);
        l2 = a * lo[m];
        rh += a * rho[m];
        a1 += a * R1[m];
        if (two) a2 += a * R2[m];
      }
      if (i + d < nr) {
        const int p = (i + d) * LB + l;
        const double b = up[o] * rcp64(lo[p] + up[p] + rho[p]);
        u2 = b * up[p];
        rh += b * rho[p];
        a1 += b * R1[p];
        if (two) a2 += b * R2[p];
      }
      nlo[q] = l2;
      nup[q] = u2;
      nrh[q] = rh;
      n1[q] = a1;
      n2[q] = a2;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int o = (2 * s + q) * LB + l;
      lo[o] = nlo[q];
      up[o] = nup[q];
      rho[o] = nrh[q];
      R1[o] = n1[q];
      if (two) R2[o] = n2[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int o = (2 * s + q) * LB + l;
    const double ir = rcp64(rho[o]);
    R1[o] *= ir;
    if (two) R2[o] *= ir;
  }
}

// US: every segment has exactly M rows.  UZ: uniform z spacing (interior
// coefficients a = c = A.hz2).
template <typename T, int M, int LB, bool US, bool UZ>
__global__ __launch_bounds__(512) void k_zsolve(T* __restrict__ x, const ZArgs A) {
  extern __shared__ double zsm[];
  const int S = A.nseg, nr = 2 * S;
  double* lo = zsm;
  double* up = lo + nr * LB;
  double* rho = up + nr * LB;
  double* R1 = rho + nr * LB;
  double* R2 = R1 + nr * LB;
  double* red = R2 + nr * LB;  // [S][LB] partial sums (singular line)
  // stretched z: the row coefficients, shared by every line, staged once
  double* cza = red + S * LB;
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
  const long line = (long)blockIdx.x * LB + l;
  x += blockIdx.y * A.batch_stride;
  const bool valid = line < A.plane;
  const bool blk0 = blockIdx.x == 0;
  const bool sing = blk0 && l == 0 && A.singular;  // line 0: lambda_x + lambda_y == 0
  const bool gen = valid && !sing;
  const bool per = A.periodic != 0;
  const long P = A.plane;
  double lam = 0.0;
  if (valid) lam = A.lamx[line % A.nx] + A.lamy[line / A.nx];
  const double ell = -lam;
  const int k0 = US ? s * M : s * A.seg_base + (s < A.seg_rem ? s : A.seg_rem);
  const int m = US ? M : A.seg_base + (s < A.seg_rem ? 1 : 0);
  const int k1 = k0 + m - 1;
  T* xs = x + (long)k0 * P + line;

  double al[M], be[M], cg[M], ta[M];
  double rlast = 0.0;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    double v = 0.0;
    if ((US || i < m) && valid) v = double(xs[(long)i * P]) * A.scale;
    al[i] = v;
    be[i] = 0.0;
    cg[i] = 0.0;
    ta[i] = 0.0;
    if (US) {
      if (i == M - 1) rlast = v;
    } else if (i == m - 1) {
      rlast = v;
    }
  }
  const double rfirst = al[0];

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
        if (i < m) acc += A.dzf[k0 + i] * al[i];
    }
    const double rbar = line_sum(acc) / A.dz_sum;
    if (sing && s == 0 && A.mean_out) A.mean_out[blockIdx.y] = rbar;
    double run = 0.0;
    if (sing) {
#pragma unroll
      for (int i = 0; i < M; ++i)
        if (i < m) {
          run += A.dzf[k0 + i] * (al[i] - rbar);
          be[i] = run;  // flux F[k+1/2]
        }
    }
    double off = line_excl(run);
    if (sing) {
#pragma unroll
      for (int i = 0; i < M; ++i) be[i] += off;
    }
    if (per) {
      // the constant flux that makes p periodic: sum_k dzc[k] F[k+1/2] = 0
      double a2 = 0.0;
      if (sing) {
#pragma unroll
        for (int i = 0; i < M; ++i)
          if (i < m) a2 += A.dzc[k0 + i] * be[i];
      }
      const double c0 = -line_sum(a2) / A.dz_sum;
      if (sing) {
#pragma unroll
        for (int i = 0; i < M; ++i) be[i] += c0;
      }
    }
    run = 0.0;
    if (sing) {
#pragma unroll
      for (int i = 0; i < M; ++i)
        if (i < m) {
          cg[i] = run;  // value p[k] relative to the segment start
          run += A.dzc[k0 + i] * be[i];
        }
    }
    off = line_excl(run);
    acc = 0.0;
    if (sing) {
#pragma unroll
      for (int i = 0; i < M; ++i)
        if (i < m) {
          cg[i] += off;
          acc += A.dzf[k0 + i] * cg[i];
        }
    }
    const double pm = line_sum(acc) / A.dz_sum;
    if (sing) {
#pragma unroll
      for (int i = 0; i < M; ++i)
        if (i < m) xs[(long)i * P] = T(cg[i] - pm);
    }
  }

  // ---- interior rows 1..m-2 of B: x_i = alpha_i + beta_i x_first + gamma_i x_last,
  //      tau = B_int^-1 1 ----
  double a1 = 0.0, b1 = 0.0, g1 = 1.0, t1 = 0.0, aL = 0.0, bL = 1.0, gL = 0.0, tL = 0.0;
  {
    double ratio = 1.0, ya = 0.0, yb = 0.0, yt = 0.0;
#pragma unroll
    for (int i = 1; i < M - 1; ++i) {
      if (US || i < m - 1) {
        double a, c;
        if (UZ) {
          a = A.hz2;
          c = A.hz2;
        } else {
          a = cza[k0 + i];
          c = czc[k0 + i];
        }
        const double sig = ell + a * ratio;
        const double iu = rcp64(c + sig);
        ratio = sig * iu;
        ya = (a * ya - al[i]) * iu;  // right-hand side of B is -r
        yb = (i == 1 ? a : a * yb) * iu;
        yt = (1.0 + a * yt) * iu;
        al[i] = ya;
        be[i] = yb;
        ta[i] = yt;
        cg[i] = c * iu;
      }
    }
    double an = 0.0, bn = 0.0, gn = 0.0, tn = 0.0;
#pragma unroll
    for (int i = M - 2; i >= 1; --i) {
      if (US || i <= m - 2) {
        const double f = cg[i];
        double gc;
        if ((US && i == M - 2) || (!US && i == m - 2)) {
          gc = f;
          aL = al[i];
          bL = be[i];
          gL = gc;
          tL = ta[i];
        } else {
          al[i] += f * an;
          be[i] += f * bn;
          ta[i] += f * tn;
          gc = f * gn;
        }
        cg[i] = gc;
        an = al[i];
        bn = be[i];
        gn = gc;
        tn = ta[i];
      }
    }
    if (US ? (M >= 3) : (m >= 3)) {
      a1 = al[1];
      b1 = be[1];
      g1 = cg[1];
      t1 = ta[1];
    }
  }

  // ---- reduced system: first and last unknown of every segment ----
  {
    const int oF = (2 * s) * LB + l, oE = (2 * s + 1) * LB + l;
    if (gen) {
      double a0, c0, aE, cE;
      if (UZ) {
        a0 = k0 == 0 ? 0.0 : A.hz2;
        c0 = A.hz2;
        aE = A.hz2;
        cE = k1 == A.nz - 1 ? 0.0 : A.hz2;
      } else {
        a0 = cza[k0];
        c0 = czc[k0];
        aE = cza[k1];
        cE = czc[k1];
      }
      lo[oF] = a0;
      up[oF] = c0 * g1;
      rho[oF] = ell * (1.0 + c0 * t1) + (k0 == 0 ? A.dlo : 0.0);
      R1[oF] = c0 * a1 - rfirst;
      lo[oE] = aE * bL;
      up[oE] = cE;
      rho[oE] = ell * (1.0 + aE * tL) + (k1 == A.nz - 1 ? A.dhi : 0.0);
      R1[oE] = aE * aL - rlast;
      // periodic: unit wrap flux entering at the first cell, leaving at the last
      R2[oF] = (per && s == 0) ? -1.0 / A.dzf[0] : 0.0;
      R2[oE] = (per && s == S - 1) ? 1.0 / A.dzf[A.nz - 1] : 0.0;
    } else {
      lo[oF] = 0.0; up[oF] = 0.0; rho[oF] = 1.0; R1[oF] = 0.0; R2[oF] = 0.0;
      lo[oE] = 0.0; up[oE] = 0.0; rho[oE] = 1.0; R1[oE] = 0.0; R2[oE] = 0.0;
    }
  }
  __syncthreads();
  red_pcr<LB>(lo, up, rho, R1, R2, per, nr, l, s);
  __syncthreads();

  if (gen) {
    const int oF = (2 * s) * LB + l, oE = (2 * s + 1) * LB + l;
    double Ft = R1[oF], Et = R1[oE];
    if (per) {
      const double xr0 = R1[l], xrn = R1[(nr - 1) * LB + l];
      const double xd0 = R2[l], xdn = R2[(nr - 1) * LB + l];
      const double fw = (xr0 - xrn) / (A.dzc_wrap - (xd0 - xdn));
      Ft += fw * R2[oF];
      Et += fw * R2[oE];
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
      if (US || i < m) {
        double v;
        if (i == 0)
          v = Ft;
        else if ((US && i == M - 1) || (!US && i == m - 1))
          v = Et;
        else
          v = al[i] + be[i] * Ft + cg[i] * Et;
        xs[(long)i * P] = T(v);
      }
    }
  }
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

template <typename T, int LB, bool US, bool UZ>
static hipError_t launch_z_shape(T* data, const ZArgs& a, int nb, hipStream_t st) {
  const int nr = 2 * a.nseg;
  const size_t shm = sizeof(double) * ((size_t)5 * nr * LB + (size_t)a.nseg * LB +
                                        (UZ ? 0 : 2 * (size_t)a.nz));
  const dim3 grid((unsigned)((a.plane + LB - 1) / LB), (unsigned)nb);
  const dim3 block((unsigned)(LB * a.nseg));
  if ((a.seg != 16 && a.seg != 8) || LB * a.nseg > 512) return hipErrorInvalidValue;
  auto kern = a.seg == 8 ? &k_zsolve<T, 8, LB, US, UZ> : &k_zsolve<T, 16, LB, US, UZ>;
  if (shm > 65536 && allow_large_lds(kern) != hipSuccess) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kern, grid, block, shm, st, data, a);
  return hipGetLastError();
}

template <typename T, int LB>
static hipError_t launch_z_lb(T* data, const ZArgs& a, int nb, hipStream_t st) {
  const bool us = a.seg_rem == 0 && a.seg_base == a.seg;
  if (us)
    return a.uniform_z ? launch_z_shape<T, LB, true, true>(data, a, nb, st)
                       : launch_z_shape<T, LB, true, false>(data, a, nb, st);
  return a.uniform_z ? launch_z_shape<T, LB, false, true>(data, a, nb, st)
                     : launch_z_shape<T, LB, false, false>(data, a, nb, st);
}

template <typename T>
static hipError_t launch_z(T* data, const ZArgs& a, int nb, hipStream_t st) {
  if (nb < 1 || nb > kMaxBatch) return hipErrorInvalidValue;
  if (a.nz == 1) {
    const dim3 grid((unsigned)((a.plane + 255) / 256), (unsigned)nb);
    hipLaunchKernelGGL((k_z1<T>), grid, dim3(256), 0, st, data, a);
    return hipGetLastError();
  }
  // LB lines x S segments per block, at most 512 lanes; a.lines picks LB
  int lb = a.lines;
  while (lb > 8 && lb * a.nseg > 512) lb /= 2;
  if (lb >= 32) return launch_z_lb<T, 32>(data, a, nb, st);
  if (lb == 16) return launch_z_lb<T, 16>(data, a, nb, st);
  if (lb * a.nseg > 512) return hipErrorInvalidValue;
  return launch_z_lb<T, 8>(data, a, nb, st);
}

hipError_t launch_zsolve_f64(double* data, const ZArgs& a, int nb, hipStream_t st) {
  return launch_z<double>(data, a, nb, st);
}
hipError_t launch_zsolve_f32(float* data, const ZArgs& a, int nb, hipStream_t st) {
  return launch_z<float>(data, a, nb, st);
}

}  // namespace vp
