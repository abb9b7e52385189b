// Marker-and-cell stencils around the Poisson solves (section 3.2: right-hand
// side of the split pressure equation and the velocity correction; section
// 3.6: the liquid-velocity extension and the interface velocity).
//
// One thread per cell (x fastest, so a wavefront reads 64 consecutive values
// of every array).  Neighbour values in x, y, z come through the L1/L2
// caches; each array is read from HBM about once.  Faces: u on i+1/2, v on
// j+1/2, w on k+1/2; a wall face (last index) has zero gradient, the face at
// -1/2 of a wall direction is implicit and zero.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace vp {

struct Nb {
  long c, xp, xm, yp, ym, zp, zm;  // neighbour offsets (-1: wall)
  int k;
};

__device__ __forceinline__ Nb neighbours(const GridArgs& g, long idx) {
  const long plane = (long)g.nx * g.ny;
  const int i = (int)(idx & (g.nx - 1));
  const int j = (int)((idx >> g.lx) & (g.ny - 1));
  const int k = (int)(idx >> (g.lx + g.ly));
  Nb n;
  n.c = idx;
  n.k = k;
  n.xp = i + 1 < g.nx ? idx + 1 : (g.bcx == 0 ? idx - (g.nx - 1) : -1);
  n.xm = i > 0 ? idx - 1 : (g.bcx == 0 ? idx + (g.nx - 1) : -1);
  n.yp = j + 1 < g.ny ? idx + g.nx : (g.bcy == 0 ? idx - (long)(g.ny - 1) * g.nx : -1);
  n.ym = j > 0 ? idx - g.nx : (g.bcy == 0 ? idx + (long)(g.ny - 1) * g.nx : -1);
  n.zp = k + 1 < g.nz ? idx + plane : (g.bcz == 0 ? idx - (long)(g.nz - 1) * plane : -1);
  n.zm = k > 0 ? idx - plane : (g.bcz == 0 ? idx + (long)(g.nz - 1) * plane : -1);
  return n;
}

// Logical block index.  Workgroups are dealt to the 8 XCDs of the chip in
// turn, each XCD with its own L2; with the remap, XCD x runs a contiguous
// range of blocks, so the rows above and below a block (its y and z
// neighbours) are mostly read by the same XCD and come from its L2.
constexpr int kXcds = 8;
__device__ __forceinline__ long logical_block(const GridArgs& g, long nblocks) {
  const long b = blockIdx.x;
  if (!g.xcd_remap) return b;
  const long per = (nblocks + kXcds - 1) / kXcds;
  return (b % kXcds) * per + b / kXcds;
}

// inverse of the face density 1 / ((rho_a + rho_b) / 2)
__device__ __forceinline__ double inv_face_rho(double ra, double rb) { return 2.0 / (ra + rb); }

// b = rho0 D[(1/rho0 - 1/rho_f) G p_hat] + (rho0/dt) (D u* - s)
__global__ __launch_bounds__(256) void k_rhs(const GridArgs g, const double* __restrict__ u,
                                              const double* __restrict__ v,
                                              const double* __restrict__ w,
                                              const double* __restrict__ ph,
                                              const double* __restrict__ rho, double rho0,
                                              const double* __restrict__ src, double dt,
                                              double* __restrict__ b, long n) {
  const long idx = logical_block(g, (n + 255) / 256) * 256 + threadIdx.x;
  if (idx >= n) return;
  const Nb nb = neighbours(g, idx);
  const double ir0 = 1.0 / rho0;
  const double p0 = ph[idx], r0 = rho[idx];
  const double idx_ = 1.0 / g.dx, idy = 1.0 / g.dy;
  const double dzf = g.dzf[nb.k];
  // flux (1/rho0 - 1/rho_f) G p_hat on the six faces of the cell
  double fxp = 0.0, fxm = 0.0, fyp = 0.0, fym = 0.0, fzp = 0.0, fzm = 0.0;
  if (nb.xp >= 0) fxp = (ir0 - inv_face_rho(r0, rho[nb.xp])) * (ph[nb.xp] - p0) * idx_;
  if (nb.xm >= 0) fxm = (ir0 - inv_face_rho(rho[nb.xm], r0)) * (p0 - ph[nb.xm]) * idx_;
  if (nb.yp >= 0) fyp = (ir0 - inv_face_rho(r0, rho[nb.yp])) * (ph[nb.yp] - p0) * idy;
  if (nb.ym >= 0) fym = (ir0 - inv_face_rho(rho[nb.ym], r0)) * (p0 - ph[nb.ym]) * idy;
  if (nb.zp >= 0) fzp = (ir0 - inv_face_rho(r0, rho[nb.zp])) * (ph[nb.zp] - p0) / g.dzc[nb.k];
  if (nb.zm >= 0) {
    const int km = nb.k > 0 ? nb.k - 1 : g.nz - 1;
    fzm = (ir0 - inv_face_rho(rho[nb.zm], r0)) * (p0 - ph[nb.zm]) / g.dzc[km];
  }
  const double divf = (fxp - fxm) * idx_ + (fyp - fym) * idy + (fzp - fzm) / dzf;
  const double um = nb.xm >= 0 ? u[nb.xm] : 0.0;
  const double vm = nb.ym >= 0 ? v[nb.ym] : 0.0;
  const double wm = nb.zm >= 0 ? w[nb.zm] : 0.0;
  const double divu = (u[idx] - um) * idx_ + (v[idx] - vm) * idy + (w[idx] - wm) / dzf;
  const double s = src ? src[idx] : 0.0;
  b[idx] = rho0 * divf + (rho0 / dt) * (divu - s);
}

// u <- u* - dt [ (1/rho0) G p + (1/rho_f - 1/rho0) G p_hat ] on the cell's
// three "plus" faces
__global__ __launch_bounds__(256) void k_correct(const GridArgs g, double* __restrict__ u,
                                                  double* __restrict__ v, double* __restrict__ w,
                                                  const double* __restrict__ p,
                                                  const double* __restrict__ ph,
                                                  const double* __restrict__ rho, double rho0,
                                                  double dt, long n) {
  const long idx = logical_block(g, (n + 255) / 256) * 256 + threadIdx.x;
  if (idx >= n) return;
  const Nb nb = neighbours(g, idx);
  const double ir0 = 1.0 / rho0;
  const double p0 = p[idx], h0 = ph[idx], r0 = rho[idx];
  if (nb.xp >= 0) {
    const double gp = (p[nb.xp] - p0) / g.dx, gh = (ph[nb.xp] - h0) / g.dx;
    u[idx] -= dt * (ir0 * gp + (inv_face_rho(r0, rho[nb.xp]) - ir0) * gh);
  }
  if (nb.yp >= 0) {
    const double gp = (p[nb.yp] - p0) / g.dy, gh = (ph[nb.yp] - h0) / g.dy;
    v[idx] -= dt * (ir0 * gp + (inv_face_rho(r0, rho[nb.yp]) - ir0) * gh);
  }
  if (nb.zp >= 0) {
    const double h = g.dzc[nb.k];
    const double gp = (p[nb.zp] - p0) / h, gh = (ph[nb.zp] - h0) / h;
    w[idx] -= dt * (ir0 * gp + (inv_face_rho(r0, rho[nb.zp]) - ir0) * gh);
  }
}

// u_1^e = u - G phi ; u_Gamma = u_1^e - q
__global__ __launch_bounds__(256) void k_extend(const GridArgs g, const double* __restrict__ u,
                                                 const double* __restrict__ v,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ phi,
                                                 const double* __restrict__ qx,
                                                 const double* __restrict__ qy,
                                                 const double* __restrict__ qz,
                                                 double* __restrict__ ue, double* __restrict__ ve,
                                                 double* __restrict__ we, double* __restrict__ ug,
                                                 double* __restrict__ vg, double* __restrict__ wg,
                                                 long n) {
  const long idx = logical_block(g, (n + 255) / 256) * 256 + threadIdx.x;
  if (idx >= n) return;
  const Nb nb = neighbours(g, idx);
  const double f0 = phi[idx];
  const double gx = nb.xp >= 0 ? (phi[nb.xp] - f0) / g.dx : 0.0;
  const double gy = nb.yp >= 0 ? (phi[nb.yp] - f0) / g.dy : 0.0;
  const double gz = nb.zp >= 0 ? (phi[nb.zp] - f0) / g.dzc[nb.k] : 0.0;
  const double a = u[idx] - gx, b = v[idx] - gy, c = w[idx] - gz;
  ue[idx] = a;
  ve[idx] = b;
  we[idx] = c;
  if (ug) {
    ug[idx] = a - qx[idx];
    vg[idx] = b - qy[idx];
    wg[idx] = c - qz[idx];
  }
}

// r = f - L_h p (FP64 residual of the defect-correction steps).  Each block
// also sums dzf[k] * p over the cells it visits (fixed order, no atomics), so
// that the weighted mean of p is known without another pass over memory.
__global__ __launch_bounds__(256) void k_residual(const GridArgs g, const double* __restrict__ f,
                                                   const double* __restrict__ p,
                                                   double* __restrict__ r,
                                                   double* __restrict__ partial, long n) {
  __shared__ double red[256];
  const double idx2 = 1.0 / (g.dx * g.dx), idy2 = 1.0 / (g.dy * g.dy);
  double acc = 0.0;
  for (long idx = (long)blockIdx.x * 256 + threadIdx.x; idx < n; idx += (long)gridDim.x * 256) {
    const Nb nb = neighbours(g, idx);
    const double p0 = p[idx];
    double lx = 0.0, ly = 0.0, lz = 0.0;
    if (nb.xp >= 0) lx += (p[nb.xp] - p0);
    if (nb.xm >= 0) lx -= (p0 - p[nb.xm]);
    if (nb.yp >= 0) ly += (p[nb.yp] - p0);
    if (nb.ym >= 0) ly -= (p0 - p[nb.ym]);
    if (nb.zp >= 0) lz += (p[nb.zp] - p0) / g.dzc[nb.k];
    if (nb.zm >= 0) {
      const int km = nb.k > 0 ? nb.k - 1 : g.nz - 1;
      lz -= (p0 - p[nb.zm]) / g.dzc[km];
    }
    r[idx] = f[idx] - (lx * idx2 + ly * idy2 + lz / g.dzf[nb.k]);
    acc += g.dzf[nb.k] * p0;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out[0] = (sum of the partial sums) / denom, one block, fixed order
__global__ __launch_bounds__(256) void k_mean_finish(const double* __restrict__ partial, int nb,
                                                      double denom, double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] / denom;
}

// grid of 256-thread blocks, rounded up to a multiple of the XCD count so
// that the remapped logical blocks cover [0, nblocks)
static inline dim3 grid_for(long n) {
  const long nb = (n + 255) / 256;
  return dim3((unsigned)((nb + kXcds - 1) / kXcds * kXcds));
}

hipError_t launch_rhs(const GridArgs& g, const double* u, const double* v, const double* w,
                      const double* phat, const double* rho, double rho0, const double* src,
                      double dt, double* b, hipStream_t st) {
  const long n = (long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k_rhs, grid_for(n), dim3(256), 0, st, g, u, v, w, phat, rho, rho0, src, dt,
                     b, n);
  return hipGetLastError();
}

hipError_t launch_correct(const GridArgs& g, double* u, double* v, double* w, const double* p,
                          const double* phat, const double* rho, double rho0, double dt,
                          hipStream_t st) {
  const long n = (long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k_correct, grid_for(n), dim3(256), 0, st, g, u, v, w, p, phat, rho, rho0,
                     dt, n);
  return hipGetLastError();
}

hipError_t launch_extend(const GridArgs& g, const double* u, const double* v, const double* w,
                         const double* phi, const double* qx, const double* qy, const double* qz,
                         double* ue, double* ve, double* we, double* ug, double* vg, double* wg,
                         hipStream_t st) {
  const long n = (long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k_extend, grid_for(n), dim3(256), 0, st, g, u, v, w, phi, qx, qy, qz, ue, ve,
                     we, ug, vg, wg, n);
  return hipGetLastError();
}

int residual_blocks(long n) {
  const long b = (n + 255) / 256;
  return (int)(b < kResidualMaxBlocks ? b : kResidualMaxBlocks);
}

hipError_t launch_residual(const GridArgs& g, const double* f, const double* p, double* r,
                           double* partial, double* mean_out, double dz_sum, hipStream_t st) {
  const long n = (long)g.nx * g.ny * g.nz;
  const int nb = residual_blocks(n);
  hipLaunchKernelGGL(k_residual, dim3(nb), dim3(256), 0, st, g, f, p, r, partial, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double denom = (double)g.nx * (double)g.ny * dz_sum;
  hipLaunchKernelGGL(k_mean_finish, dim3(1), dim3(256), 0, st, partial, nb, denom, mean_out);
  return hipGetLastError();
}

}  // namespace vp
