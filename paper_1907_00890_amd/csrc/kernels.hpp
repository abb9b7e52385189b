// Host-side launchers of the HIP kernels (internal to libvofpoisson).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "bc.hpp"
#include "limits.hpp"

namespace vp {

// Tile of hardware block h of a one-dimensional grid of G blocks.  Blocks are
// dispatched to the eight XCDs in turn (h % 8), each XCD with its own L2; here
// XCD x takes the contiguous tiles [x G/8, (x+1) G/8) (one more for the first
// G % 8 XCDs) in order, so that neighbouring tiles whose rows share 128-byte
// cache lines (tiles narrower than a line) are read through one L2, one after
// the other, instead of by two XCDs at once.  A bijection of [0, G).
__device__ __forceinline__ unsigned xcd_tile(unsigned h, unsigned G) {
  const unsigned q = G / 8, r = G % 8, x = h % 8;
  return x * q + (x < r ? x : r) + h / 8;
}

// (tile, layer) of hardware block (bx, by) of a two-dimensional grid of gx
// tiles by gy layers, for passes that walk the layers in order: XCD x takes
// the layers x, x+8, x+16, ... whole, their tiles in order, so neighbouring
// tiles of a layer share one L2 and the layers still run in their order.  The
// last gy % 8 layers keep their ids.  A bijection of the grid.
__device__ __forceinline__ uint2 xcd_layer(unsigned bx, unsigned by, unsigned gx, unsigned gy) {
  const unsigned h = bx + gx * by;
  if (h >= (gy / 8) * 8 * gx) return make_uint2(bx, by);
  const unsigned j = h / 8, L = ((j / gx) * 8 + h % 8) * gx + j % gx;
  return make_uint2(L % gx, L / gx);
}

// 1/x for a positive normal x: hardware reciprocal estimate refined by two
// Newton-Raphson steps (r <- r + r (1 - x r)), accurate to about one ulp
// (five instructions against about ten for an IEEE division).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Raise a kernel's dynamic-LDS limit to the 160 KB of a gfx950 CU (for
// launches above 64 KB); done once per kernel and device (kernels of one
// signature are distinct entries: the key is the kernel's address).
inline hipError_t allow_large_lds_fn(const void* kernel) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, hipError_t> done;
  int dev = 0;
  const hipError_t ge = hipGetDevice(&dev);
  if (ge != hipSuccess) return ge;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(dev, kernel);
  const auto it = done.find(key);
  if (it != done.end()) return it->second;
  const hipError_t e =
      hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  done.emplace(key, e);
  return e;
}
template <typename K>
inline hipError_t allow_large_lds(K* kernel) {
  return allow_large_lds_fn(reinterpret_cast<const void*>(kernel));
}

// Up to kMaxBatch independent fields go through one launch of each pass: the
// batch member is blockIdx.y (x and z passes) or folded into the plane index
// (y pass, the spectra of a batch are consecutive).  Caller-owned fields are
// passed as a table of pointers, by value in the kernel arguments.
template <typename T>
struct Batch {
  T* p[kMaxBatch];
};
template <typename T>
inline Batch<T> batch_of(T* const* ptrs, int n) {
  Batch<T> b{};
  for (int i = 0; i < n && i < kMaxBatch; ++i) b.p[i] = ptrs[i];
  return b;
}

// transforms_x.hip, transforms_y.hip ------------------------------------------
// tab layout per direction and precision, (cos, sin) pairs: of 2 pi k/N for
// k < N, then of pi m/(2N) for m <= N/2 (one 2-vector load per twiddle).
int ypass_tile_cols(int nx, int ny);
// Partial sums of the mixed chain's x passes: kNormSlots doubles per x
// block of a batch member (layout in transforms_x.hip).
constexpr int kNormSlots = 4;

// Geometry of the mixed chain's x passes: plane widths for the weighted sums,
// and the stencil of the residual mode of the x forward pass, which reads
// f - m - L_h p (p: current iterate of each member, m: mean[b], or 0 where
// mean is null) in place of f.
struct ResidualArgs {
  Batch<const double> p;
  const double* mean;
  const double* dzf;   // nz
  const double* dzc;   // nz, as GridArgs::dzc
  double idx2, idy2;   // 1 / dx^2, 1 / dy^2
  int ny, nz;
  int perx, pery, perz;  // periodic directions
  int outflow;           // as GridArgs::outflow
};

// Options of the FP32 passes of the mixed-precision chain (FP32 spectra in
// HBM, FP64 arithmetic, LDS and twiddle tables inside every pass):
//   sub      : x inverse with accumulation subtracts sub[b] from member b's
//              result (the weighted mean of the previous iterate);
//   skip     : per-member flags; a member whose flag is set is left untouched
//              (its blocks return at once); null: every member runs;
//   norms    : x passes write their per-block partial sums (kNormSlots each);
//   geo      : x passes of the mixed chain (required there);
//   residual : x forward in residual mode;
//   nzm      : z-planes per member (y passes: member = plane / nzm);
//   lines    : y passes: column pairs per block (a power of two; 0: default).
struct PassOpts {
  const double* sub = nullptr;
  const int* skip = nullptr;
  double* norms = nullptr;
  const ResidualArgs* geo = nullptr;
  bool residual = false;
  int nzm = 0;
  int lines = 0;
};

// x passes: `in`/`out` hold nb caller fields; the spectra of batch member b
// start at b * stride of the workspace.  pt: values per thread of the radix
// schedule of every transform pass (16: radix-16 passes, 8: radix-8).
hipError_t launch_xfwd_f64(const Batch<const double>& in, int nb, double* out, long ostride,
                           int nx, int bc, long nrows, const double* tab, int pt,
                           hipStream_t st);
hipError_t launch_xinv_f64(const double* in, long istride, const Batch<double>& out, int nb,
                           int nx, int bc, long nrows, const double* tab, int pt,
                           hipStream_t st);
hipError_t launch_xfwd_f32(const Batch<const double>& in, int nb, float* out, long ostride,
                           int nx, int bc, long nrows, const double* tab, int pt,
                           const PassOpts& o, hipStream_t st);
// accum: out += result - o.sub[b] for batch member b (o.sub may be null)
hipError_t launch_xinv_f32(const float* in, long istride, const Batch<double>& out, int nb,
                           int nx, int bc, long nrows, bool accum, const double* tab, int pt,
                           const PassOpts& o, hipStream_t st);
// blocks per member of an x pass (the norms partial sums of the x inverse)
long xpass_blocks(int nx, int bc, int pt, long nrows);
// y passes over nplanes consecutive z-planes (nz * batch)
hipError_t launch_y_f64(double* data, int nx, int ny, int nplanes, int bc, bool fwd,
                        const double* tab, int pt, int lines, hipStream_t st);
hipError_t launch_y_f32(float* data, int nx, int ny, int nplanes, int bc, bool fwd,
                        const double* tab, int pt, const PassOpts& o, hipStream_t st);

// spectral z pass for a uniform z grid with nz a transform length (2^k in
// [8, 1024], 3 * 2^k in [24, 768] or 5 * 2^k in [40, 640]):
// forward real DFT / DCT-II / DST-II along z, division by the 3-D eigenvalue,
// inverse, in one pass (transforms_z.hip)
struct ZSpecArgs {
  int nx, ny, nz;
  int bcz;             // BC_P, BC_N or BC_D
  double scale;        // 1 / (nx * ny * nz)
  const double* lamx;  // eigenvalue per packed x, y, z position
  const double* lamy;
  const double* lamz;
  long batch_stride;
  double* mean_out;    // removed mean of member b at [b], may be null
  int lines;           // column pairs per block (a power of two; 0: the y pass's width)
};
hipError_t launch_zspec_f64(double* data, const ZSpecArgs& a, const double* tab, int pt, int nb,
                            hipStream_t st);
hipError_t launch_zspec_f32(float* data, const ZSpecArgs& a, const double* tab, int pt, int nb,
                            const int* skip, hipStream_t st);

// zsolve.hip -----------------------------------------------------------------
struct ZArgs {
  long plane;          // nx * ny lines
  int nx;              // for the (cx, cy) split of a line index
  int nz;
  int seg;             // segment length bound M (16; 8 on stretched grids with nz <= 512)
  int lines;           // lines per block (8, 16 or 32; capped so lines * nseg <= 512)
  int nseg;            // S segments per line
  int seg_base;        // nz / S
  int seg_rem;         // nz % S (first seg_rem segments are one longer)
  int periodic;        // z periodic
  int singular;        // no outflow end anywhere: line (0, 0) is singular
  double dlo, dhi;     // outflow at z- / z+: 2 / dz^2 of the end cell added to the
                       // diagonal of -(A + lambda); 0 at a wall
  double scale;        // 1 / (nx * ny)
  double dz_sum;       // sum of dzf
  const double* lamx;  // eigenvalue per packed x position
  const double* lamy;
  double dzc_wrap;     // centre distance across the wrap face (periodic z)
  int uniform_z;       // all dzf equal: interior coefficients are hz2
  double hz2;          // 1 / dz^2 of a uniform z grid
  const double* za;    // sub-diagonal of the row-scaled z operator (wall form: za[0] = 0)
  const double* zc;    // super-diagonal (wall form: zc[nz-1] = 0)
  const double* dzf;
  const double* dzc;   // centre distance across face k+1/2 (wrap at nz-1 if periodic)
  double* mean_out;    // removed weighted mean of batch member b at [b] (diagnostic), may be null
  long batch_stride;   // elements between the spectra of consecutive batch members
  const int* skip;     // per-member flags: set = leave the member untouched (may be null)
};
hipError_t launch_zsolve_f64(double* data, const ZArgs& a, int nb, hipStream_t st);
hipError_t launch_zsolve_f32(float* data, const ZArgs& a, int nb, hipStream_t st);

// stencils.hip ---------------------------------------------------------------
struct GridArgs {
  int nx, ny, nz;
  int txp;             // largest power of two dividing nx (tile widths divide it)
  int kc;              // z-planes marched by one stencil block
  int tiled;           // right-hand side on LDS-staged 64 x tiled tiles (8 or 16 rows) where
                       // they fit; 0: plain 64 x 4 tiles
  int bcx, bcy, bcz;   // 0 periodic, 1 wall or outflow
  int outflow;         // bit 2d: outflow at the lower end of direction d (x, y, z),
                       // bit 2d+1: at the upper end
  double dx, dy;
  const double* dzf;   // nz
  const double* dzc;   // nz (last entry: wrap distance when z is periodic, dzf[nz-1]
                       // -- the distance to the mirrored ghost -- with an outflow at z+)
};
hipError_t launch_rhs(const GridArgs& g, const double* u, const double* v, const double* w,
                      const double* phat, const double* rho, double rho0, const double* src,
                      double dt, double* b, hipStream_t st);
hipError_t launch_correct(const GridArgs& g, double* u, double* v, double* w, const double* p,
                          const double* phat, const double* rho, double rho0, double dt,
                          hipStream_t st);
hipError_t launch_extend(const GridArgs& g, const double* u, const double* v, const double* w,
                         const double* phi, const double* qx, const double* qy, const double* qz,
                         double* ue, double* ve, double* we, double* ug, double* vg, double* wg,
                         hipStream_t st);
hipError_t launch_step_epilogue(const GridArgs& g, double* u, double* v, double* w, const double* p,
                                const double* phat, const double* rho, double rho0, double dt,
                                const double* phi, const double* qx, const double* qy,
                                const double* qz, double* ue, double* ve, double* we, double* ug,
                                double* vg, double* wg, hipStream_t st);
// interface terms s, q from the volume fraction C and the mass flux mdot
// (Youngs gradient of C; one z-marching pass, g.kc planes per block of
// kInterfaceThreads threads on a min(txp, 64) x (kInterfaceThreads / width)
// tile)
constexpr int kInterfaceThreads = 512;
hipError_t launch_interface(const GridArgs& g, const double* C, const double* mdot, double rho1,
                            double rho2, double rho_e, double* s, double* qx, double* qy,
                            double* qz, hipStream_t st);
// The interface terms fused into the step's first and last passes (the
// march of launch_interface carrying a second stencil):
//   launch_rhs_interface      : s (written) and the pressure right-hand side b
//                               = launch_rhs with src = s; reads u, v, w, ph, rho;
//   launch_epilogue_interface : launch_step_epilogue with q the face means of
//                               a = (mdot / rho_e) n, in place on uo, vo, wo;
//                               ue.. optional, ug.. required.
struct IfStepArgs {
  const double* u = nullptr;  // u*, v*, w* (right-hand side)
  const double* v = nullptr;
  const double* w = nullptr;
  double* uo = nullptr;       // u*, v*, w* in, u^{n+1} out (epilogue)
  double* vo = nullptr;
  double* wo = nullptr;
  const double* ph = nullptr;
  const double* rho = nullptr;
  double rho0 = 1.0, dt = 1.0;
  double* b = nullptr;
  const double* p = nullptr;
  const double* phi = nullptr;
  double *ue = nullptr, *ve = nullptr, *we = nullptr;
  double *ug = nullptr, *vg = nullptr, *wg = nullptr;
};
hipError_t launch_rhs_interface(const GridArgs& g, const double* C, const double* mdot,
                                double rho1, double rho2, double* s, const IfStepArgs& a,
                                hipStream_t st);
hipError_t launch_epilogue_interface(const GridArgs& g, const double* C, const double* mdot,
                                     double rho_e, const IfStepArgs& a, hipStream_t st);
// Faces at -1/2 of a lower outflow end in direction dir (0 x, 1 y, 2 z):
// their velocities uf (and ue on them, uef) as one plane; see stencils.hip.
enum : int { LF_RHS = 0, LF_CORRECT = 1, LF_EXTEND = 2, LF_STEP = 3 };
hipError_t launch_lower_faces(const GridArgs& g, int mode, int dir, double* uf, double* uef,
                              double* b, const double* p, const double* ph, const double* rho,
                              double rho0, double dt, const double* phi, hipStream_t st);
// advect.hip: VoF advection of section 3.1 (directional split, MTHINC flux,
// volume deflation).  sweep 0: x sweep C -> out; 1: y sweep out -> work;
// 2: z sweep work -> out with the final correction (C* read back from out).
// g.txp sets the tile width (one thread per cell, 256 per block).
// lo[d]: the interface velocity on the faces at -1/2 of a lower outflow end
// in direction d (a plane, as for launch_lower_faces), null elsewhere.
hipError_t launch_advect(const GridArgs& g, const double* C, const double* ug, const double* vg,
                         const double* wg, const double* const* lo, double dt, double beta,
                         int deflation, double* work, double* out, int sweep, hipStream_t st);
int stencil_blocks(const GridArgs& g);
int rhs_blocks(const GridArgs& g);  // blocks of one launch_rhs
int stencil_default_planes(int nx, int ny, int nz);
// Defect-correction control of the mixed chain, per member b of a batch of
// nb (state: 4 doubles per member, flags: one int per member).
// dc_update reduces the x-pass partial sums
// of step `step` (0 = the first FP32 solve; nblk blocks per member), writes
// pmean[b] (weighted mean of the iterate: sum dzf p / denom) and, at step 0,
// fmean[b] (of f) and a cleared flag[b]; from step 1 on it sets flag[b] once
// the error estimate
// 2^-23 (gain |r| + |e|) / |p| of the step is at most tol (tol <= 0: never).
hipError_t launch_dc_update(const double* norms, long nblk, int nb, int step, double tol,
                            double gain, double denom, double* state, int* flags, double* pmean,
                            double* fmean, hipStream_t st);

}  // namespace vp
