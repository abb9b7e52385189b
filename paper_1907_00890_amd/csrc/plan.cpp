// Plan, workspace and C entry points of libvofpoisson (see include/vofpoisson.h).
//
// Spectral solve (the constant-coefficient direct solver of section 3.2, used
// again for the Stefan potential of section 3.6):
//   x pass (forward)  -> y pass (forward) -> z tridiagonal pass
//   -> y pass (inverse) -> x pass (inverse)
// The forward transforms are unnormalised; the z pass scales by 1/(nx*ny)
// and the inverse transforms return N times their input, so the chain is
// exactly the inverse operator on the zero-mean subspace (the inverse itself
// when an outflow end makes the operator non-singular).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bc.hpp"
#include "kernels.hpp"
#include "vofpoisson.h"

namespace {

thread_local std::string g_last_error;

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? VP_ENOMEM : VP_EHIP;
}

#define VP_HIP(call, what)                       \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

enum KernelClass {
  K_XFWD = 0, K_YFWD, K_Z, K_YINV, K_XINV,
  K_XFWD32, K_YFWD32, K_Z32, K_YINV32, K_XINV32,
  K_RESIDUAL, K_RHS, K_CORRECT, K_EXTEND, K_EPILOGUE, K_INTERFACE,
  K_ADV_X, K_ADV_Y, K_ADV_Z, K_NCLASS
};
static_assert(K_NCLASS <= VP_NUM_KERNEL_CLASSES, "kernel classes of the C interface");
const char* const kClassNames[K_NCLASS] = {
    "x_forward", "y_forward", "z_solve", "y_inverse", "x_inverse",
    "x_forward_f32", "y_forward_f32", "z_solve_f32", "y_inverse_f32", "x_inverse_f32",
    "x_forward_residual_f32", "rhs_assembly", "correction", "extension", "step_epilogue",
    "interface_terms",
    "advect_x", "advect_y", "advect_z"};

// Twiddle table of one direction, (cos, sin) pairs: of 2 pi k/N for k < N,
// then of pi m/(2N) for m <= N/2 (the DCT post/pre rotation).  For a wall at
// one end and an outflow at the other (the quarter-wave transform, a complex
// FFT of length H = N/2): of 2 pi j/H for j < H, of pi (4e+1)/(4N) for
// e < H, of pi k/N for k < H.  Both layouts have the same size.
std::vector<double> make_table(int n, int bc) {
  std::vector<double> t(2 * n + 2 * (n / 2 + 1), 0.0);
  const double pi = 3.14159265358979323846264338327950288;
  auto put = [&](int pair, double angle) {
    t[2 * pair] = std::cos(angle);
    t[2 * pair + 1] = std::sin(angle);
  };
  if (bc == vp::BC_ND || bc == vp::BC_DN) {
    const int h = n / 2;
    for (int j = 0; j < h; ++j) put(j, 2.0 * pi * j / h);
    for (int e = 0; e < h; ++e) put(h + e, pi * (4.0 * e + 1.0) / (4.0 * n));
    for (int k = 0; k < h; ++k) put(2 * h + k, pi * k / n);
    return t;
  }
  for (int k = 0; k < n; ++k) put(k, 2.0 * pi * k / n);
  for (int m = 0; m <= n / 2; ++m) put(n + m, pi * m / (2.0 * n));
  return t;
}

// Eigenvalue of the 1-D second difference for every packed coefficient
// position: periodic -(4/h^2) sin^2(pi m/n) (packed real DFT order), walls
// -(4/h^2) sin^2(pi c/(2n)) (cosine mode c), outflow at both ends
// -(4/h^2) sin^2(pi (n-c)/(2n)) = -(4/h^2) cos^2(pi c/(2n)) (sine mode n-1-c),
// a wall and an outflow -(4/h^2) sin^2(pi (2c+1)/(4n)) (quarter-wave mode c).
std::vector<double> make_lambda(int n, double h, int bc) {
  const double pi = 3.14159265358979323846264338327950288;
  std::vector<double> l(n);
  for (int c = 0; c < n; ++c) {
    double s;
    if (bc == vp::BC_P) {
      const int m = c == 0 ? 0 : (c == 1 ? n / 2 : c / 2);
      s = std::sin(pi * m / n);
    } else if (bc == vp::BC_N) {
      s = std::sin(pi * c / (2.0 * n));
    } else if (bc == vp::BC_D) {
      s = std::cos(pi * c / (2.0 * n));
    } else {
      s = std::sin(pi * (2.0 * c + 1.0) / (4.0 * n));
    }
    l[c] = -4.0 / (h * h) * s * s;
  }
  return l;
}

// segment length of the partitioned z solve (8 or 16 rows): S = ceil(nz / M)
// segments, the first nz % S one row longer
void set_z_segment(vp::ZArgs& Z, int seg) {
  Z.seg = seg;
  Z.nseg = (Z.nz + seg - 1) / seg;
  Z.seg_base = Z.nz / Z.nseg;
  Z.seg_rem = Z.nz % Z.nseg;
}

}  // namespace

// Spectrum slot of poisson_solve_noalloc: a static device array (every GPU
// the library runs on holds its own copy until the process ends).  Host code
// never uses its name as an address: the per-device address comes from
// hipGetSymbolAddress, taken once per device at set-up (plan creation, or
// the entry point's first call on a device) with that device current.
static_assert(VP_NOALLOC_MAX_POINTS == (1 << 23), "size of the static spectrum slot");
static __device__ __align__(256) double scratch[VP_NOALLOC_MAX_POINTS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on `device` (the current device), or null
// with the HIP error kept for poisson_strerror
double* scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) {
    g_last_error = "noalloc scratch: device index out of range";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      g_last_error = std::string("noalloc scratch: hipGetSymbolAddress: ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[device];
}

}  // namespace

struct poisson_plan {
  int nx = 0, ny = 0, nz = 0;
  int bc[3] = {0, 0, 0};  // transform codes of x, y, z (vp::BC_*)
  char ends[6] = {};      // 'P' / 'N' / 'D' at x-, x+, y-, y+, z-, z+
  bool singular = true;   // no outflow end: the constants are the null space
  int precision = 0, max_batch = 1, dc_steps = 1;
  int x_pt = 16, y_pt = 16;  // radix schedules of the x and y passes (tuning knobs)
  int y_lines = 0;           // column pairs per y block (0: the default width)
  double dx = 0, dy = 0, dz_sum = 0;
  int device = 0;
  long long bytes = 0;
  std::vector<void*> allocs;

  // twiddle tables (FP64; the mixed chain computes in FP64 too and stores FP32)
  double *tabx64 = nullptr, *taby64 = nullptr;
  double *lamx = nullptr, *lamy = nullptr, *za = nullptr, *zc = nullptr;
  // spectral z pass (uniform z, nz a power of two in [8, 1024])
  double *lamz = nullptr, *tabz64 = nullptr;
  vp::ZSpecArgs zs{};
  int z_spec_ok = 0, z_spec = 0, z_pt = 16;
  double *dzf = nullptr, *dzc = nullptr, *mean = nullptr;
  double* work64 = nullptr;
  float* work32 = nullptr;
  // mixed-precision correction control: per-member state, flags, the x-pass
  // partial sums, the stencil and plane widths of the FP32 x passes, and the
  // noise gain of the error estimate
  double* dc_state = nullptr;
  int* dc_flags = nullptr;
  double* dc_norms = nullptr;
  double dc_tol = 1e-11;
  vp::ResidualArgs rgeo{};
  double noise_gain = 0.0;

  vp::ZArgs z{};
  vp::GridArgs g{};   // marching stencils (right-hand side)
  vp::GridArgs gs{};  // streaming stencils (correction, extension)
  vp::GridArgs ge{};  // fused step epilogue
  vp::GridArgs gi{};  // interface terms

  // optional per-launch timing (HIP events on the caller's stream)
  struct Mark {
    int cls;
    hipEvent_t a, b;
  };
  unsigned profiling = 0;  // bit c: bracket launches of kernel class c
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  hipEvent_t event() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
      e = pool.back();
      pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }

  long npts() const { return (long)nx * ny * nz; }

  template <typename T>
  int alloc(T** p, size_t count, const char* what) {
    void* q = nullptr;
    VP_HIP(hipMalloc(&q, count * sizeof(T)), what);
    allocs.push_back(q);
    bytes += (long long)(count * sizeof(T));
    *p = static_cast<T*>(q);
    return VP_OK;
  }
  template <typename T>
  int upload(T** p, const std::vector<T>& h, const char* what) {
    int st = alloc(p, h.size(), what);
    if (st) return st;
    VP_HIP(hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), what);
    return VP_OK;
  }
  void release() {
    for (void* q : allocs) (void)hipFree(q);
    allocs.clear();
    for (auto& m : marks) {
      (void)hipEventDestroy(m.a);
      (void)hipEventDestroy(m.b);
    }
    marks.clear();
    for (auto e : pool) (void)hipEventDestroy(e);
    pool.clear();
  }
};

namespace {

// Launch `call` on stream st; with profiling on, bracket it with two events.
#define VP_LAUNCH(P, cls, call, what, st)                                 \
  do {                                                                    \
    hipEvent_t a_ = nullptr, b_ = nullptr;                                \
    const bool prof_ = ((P)->profiling >> (cls)) & 1u;                    \
    if (prof_) {                                                          \
      a_ = (P)->event();                                                  \
      b_ = (P)->event();                                                  \
      if (a_) (void)hipEventRecord(a_, st);                               \
    }                                                                     \
    VP_HIP((call), what);                                                 \
    if (prof_ && a_ && b_) {                                              \
      (void)hipEventRecord(b_, st);                                       \
      (P)->marks.push_back({cls, a_, b_});                                \
    }                                                                     \
  } while (0)

// Noise gain of the mixed chain's error estimate: the RMS over z modes of
// 1/|lambda| for the worst (kx, ky) line,
//   G^2 = (1/nz) sum_{k: mu_k > 0} 1/mu_k^2  +  [z null mode] 1/(nz s^2),
// mu_k the eigenvalues of the z operator -W^-1 S (W = diag(dzf), f below;
// c: centre distances as in plan_init) and s the smallest non-zero
// |lambda_x| + |lambda_y| (a line with s > 0 has 1/(s + mu_k)^2 <= 1/mu_k^2
// for mu_k > 0 and 1/s^2 for a null mode).  The sum is the squared Frobenius
// norm of the pseudo-inverse of the symmetric form M = W^-1/2 (-S) W^-1/2,
// taken one column at a time with tridiagonal solves: where M is singular
// (no outflow at a z end) its null vector v ~ sqrt(dzf) is projected out of
// e_j, the first unknown is pinned to 0 (which drops the periodic couplings,
// all through unknown 0) and v is projected out of the solution.
double mixed_noise_gain(const std::vector<double>& f, const std::vector<double>& c, bool zper,
                        bool lo_out, bool hi_out, const std::vector<double>& lx,
                        const std::vector<double>& ly) {
  const int nz = (int)f.size();
  std::vector<double> d(nz, 0.0), e(nz, 0.0);  // diagonal, coupling k <-> k+1
  for (int k = 0; k < nz; ++k) {
    double a = 0.0;
    if (k > 0) a += 1.0 / c[k - 1];
    else if (zper) a += 1.0 / c[nz - 1];
    if (k + 1 < nz) a += 1.0 / c[k];
    else if (zper) a += 1.0 / c[nz - 1];
    if (k == 0 && lo_out) a += 2.0 / f[0];
    if (k == nz - 1 && hi_out) a += 2.0 / f[nz - 1];
    d[k] = a / f[k];
    if (k + 1 < nz) e[k] = -1.0 / (c[k] * std::sqrt(f[k] * f[k + 1]));
  }
  const bool sing = !lo_out && !hi_out;
  std::vector<double> v(nz);
  double vs = 0.0;
  for (int k = 0; k < nz; ++k) vs += f[k];
  for (int k = 0; k < nz; ++k) v[k] = std::sqrt(f[k] / vs);
  // tridiagonal solve of rows/columns k0..nz-1 of M (Thomas, no pivoting:
  // M restricted there is symmetric positive definite)
  const int k0 = sing ? 1 : 0;
  std::vector<double> cp(nz, 0.0), x(nz, 0.0), rhs(nz, 0.0);
  double sum = 0.0;
  for (int j = 0; j < nz; ++j) {
    for (int k = 0; k < nz; ++k) rhs[k] = (k == j ? 1.0 : 0.0) - (sing ? v[k] * v[j] : 0.0);
    x[0] = 0.0;
    double den = 1.0;
    for (int k = k0; k < nz; ++k) {
      const double lo = k > k0 ? e[k - 1] : 0.0;
      den = d[k] - (k > k0 ? lo * cp[k - 1] : 0.0);
      cp[k] = k + 1 < nz ? e[k] / den : 0.0;
      x[k] = (rhs[k] - (k > k0 ? lo * x[k - 1] : 0.0)) / den;
    }
    for (int k = nz - 2; k >= k0; --k) x[k] -= cp[k] * x[k + 1];
    if (sing) {
      double dot = 0.0;
      for (int k = 0; k < nz; ++k) dot += v[k] * x[k];
      for (int k = 0; k < nz; ++k) x[k] -= dot * v[k];
    }
    for (int k = 0; k < nz; ++k) sum += x[k] * x[k];
  }
  double g2 = sum / nz;
  if (sing) {
    auto min_pos = [](const std::vector<double>& l, double& mn) {
      double mp = 0.0;
      mn = std::fabs(l[0]);
      for (double t : l) {
        const double a = std::fabs(t);
        mn = std::min(mn, a);
        if (a > 0.0 && (mp == 0.0 || a < mp)) mp = a;
      }
      return mp;
    };
    double mx = 0.0, my = 0.0;
    const double px = min_pos(lx, mx), py = min_pos(ly, my);
    double smin = 0.0;
    if (px > 0.0) smin = px + my;
    if (py > 0.0 && (smin == 0.0 || py + mx < smin)) smin = py + mx;
    if (smin > 0.0) g2 += 1.0 / (nz * smin * smin);
  }
  return std::sqrt(g2);
}

int plan_init(poisson_plan* P, const double* dz) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  int st;
  // tables
  const std::vector<double> tx = make_table(nx, P->bc[0]), ty = make_table(ny, P->bc[1]);
  if ((st = P->upload(&P->tabx64, tx, "table x"))) return st;
  if ((st = P->upload(&P->taby64, ty, "table y"))) return st;
  const std::vector<double> lx = make_lambda(nx, P->dx, P->bc[0]);
  const std::vector<double> ly = make_lambda(ny, P->dy, P->bc[1]);
  if ((st = P->upload(&P->lamx, lx, "lambda x"))) return st;
  if ((st = P->upload(&P->lamy, ly, "lambda y"))) return st;

  // z grid: centre distances and the row-scaled tridiagonal coefficients
  const bool zper = P->bc[2] == vp::BC_P;
  std::vector<double> f(dz, dz + nz), c(nz, 0.0), a(nz, 0.0), cc(nz, 0.0);
  double sum = 0.0;
  for (int k = 0; k < nz; ++k) sum += f[k];
  for (int k = 0; k + 1 < nz; ++k) c[k] = 0.5 * (f[k] + f[k + 1]);
  if (zper) c[nz - 1] = 0.5 * (f[nz - 1] + f[0]);
  else if (P->ends[5] == 'D') c[nz - 1] = f[nz - 1];  // to the mirrored ghost of the outflow face
  else c[nz - 1] = 1.0;  // unused (wall)
  // wall form of the operator; a periodic z adds the wrap face through one
  // flux unknown inside the z kernel (distance c[nz-1])
  for (int k = 0; k < nz; ++k) {
    if (k > 0) a[k] = 1.0 / (f[k] * c[k - 1]);
    if (k + 1 < nz) cc[k] = 1.0 / (f[k] * c[k]);
  }
  P->dz_sum = sum;
  if ((st = P->upload(&P->dzf, f, "dzf"))) return st;
  if ((st = P->upload(&P->dzc, c, "dzc"))) return st;
  if ((st = P->upload(&P->za, a, "za"))) return st;
  if ((st = P->upload(&P->zc, cc, "zc"))) return st;
  if ((st = P->alloc(&P->mean, 3 * vp::kMaxBatch, "mean"))) return st;
  VP_HIP(hipMemset(P->mean, 0, 3 * vp::kMaxBatch * sizeof(double)), "mean init");

  // one spectrum slot per batch member
  const size_t n = (size_t)P->npts() * P->max_batch;
  if ((st = P->alloc(&P->work64, n, "workspace"))) return st;
  if (P->precision == VP_PRECISION_MIXED) {
    if ((st = P->alloc(&P->work32, n, "workspace f32"))) return st;
    if ((st = P->alloc(&P->dc_state, 4 * vp::kMaxBatch, "dc state"))) return st;
    if ((st = P->alloc(&P->dc_flags, vp::kMaxBatch, "dc flags"))) return st;
    // kNormSlots partial sums per x block; a block owns at least four rows
    // (ny * nz is a multiple of 8), so ny * nz doubles per member hold them
    if ((st = P->alloc(&P->dc_norms, (size_t)P->ny * P->nz * P->max_batch, "dc norms"))) return st;
    P->noise_gain = mixed_noise_gain(f, c, zper, P->ends[4] == 'D', P->ends[5] == 'D', lx, ly);
  }

  // z launch geometry: S segments of at most 16 rows (S <= 64)
  vp::ZArgs& Z = P->z;
  Z.plane = (long)nx * ny;
  Z.nx = nx;
  Z.nz = nz;
  // segments of at most 16 rows; 8 on stretched grids with nz <= 512 (fewer
  // registers per lane for the row coefficients: measured 549 against 588 us
  // at 512 x 512 x 256); a tuning knob, tried by the autotuner
  {
    bool uni = true;
    for (int k = 1; k < nz; ++k) uni = uni && f[k] == f[0];
    set_z_segment(Z, (!uni && nz <= 512) ? 8 : 16);
  }
  Z.lines = 16;
  Z.periodic = zper ? 1 : 0;
  Z.singular = P->singular ? 1 : 0;
  Z.dlo = P->ends[4] == 'D' ? 2.0 / (f[0] * f[0]) : 0.0;
  Z.dhi = P->ends[5] == 'D' ? 2.0 / (f[nz - 1] * f[nz - 1]) : 0.0;
  Z.dzc_wrap = zper ? c[nz - 1] : 0.0;
  // a uniform grid (bitwise equal widths) lets the z kernel use one constant
  // coefficient; za / zc hold exactly that value in the interior
  Z.uniform_z = 1;
  for (int k = 1; k < nz; ++k)
    if (f[k] != f[0]) Z.uniform_z = 0;
  Z.hz2 = nz > 1 ? cc[0] : 0.0;
  if (Z.uniform_z) {
    for (int k = 1; k + 1 < nz; ++k)
      if (a[k] != Z.hz2 || cc[k] != Z.hz2) Z.uniform_z = 0;
  }
  Z.scale = 1.0 / ((double)nx * (double)ny);
  Z.dz_sum = sum;
  Z.lamx = P->lamx;
  Z.lamy = P->lamy;
  Z.za = P->za;
  Z.zc = P->zc;
  Z.dzf = P->dzf;
  Z.dzc = P->dzc;
  Z.mean_out = P->mean;
  Z.batch_stride = P->npts();

  // a uniform z line of a transform length is diagonalised exactly by the
  // real DFT (periodic), DCT-II (walls) or DST-II (outflow at both ends) of
  // the x and y passes; a wall at one end and an outflow at the other keeps
  // the tridiagonal pass
  P->z_spec_ok = Z.uniform_z && vp::fft_length(nz) &&
                 P->bc[2] <= vp::BC_D;
  if (P->z_spec_ok) {
    const std::vector<double> tz = make_table(nz, P->bc[2]);
    if ((st = P->upload(&P->tabz64, tz, "table z"))) return st;
    if ((st = P->upload(&P->lamz, make_lambda(nz, f[0], P->bc[2]), "lambda z"))) return st;
    vp::ZSpecArgs& A = P->zs;
    A.nx = nx;
    A.ny = ny;
    A.nz = nz;
    A.bcz = P->bc[2];
    A.scale = 1.0 / ((double)nx * (double)ny * (double)nz);
    A.lamx = P->lamx;
    A.lamy = P->lamy;
    A.lamz = P->lamz;
    A.batch_stride = P->npts();
    A.mean_out = P->mean;
    P->z_spec = 1;
  }

  vp::GridArgs& G = P->g;
  G.nx = nx; G.ny = ny; G.nz = nz;
  G.txp = nx & -nx;
  G.bcx = P->bc[0] == vp::BC_P ? 0 : 1;
  G.bcy = P->bc[1] == vp::BC_P ? 0 : 1;
  G.bcz = P->bc[2] == vp::BC_P ? 0 : 1;
  G.outflow = 0;
  for (int e = 0; e < 6; ++e)
    if (P->ends[e] == 'D') G.outflow |= 1 << e;
  G.dx = P->dx; G.dy = P->dy;
  G.dzf = P->dzf; G.dzc = P->dzc;
  G.kc = vp::stencil_default_planes(nx, ny, nz);
  G.tiled = 8;
  // the correction and the extension alone run as the epilogue's kinds on
  // the same LDS-staged tiles where they fit, one plane per block
  P->gs = G;
  P->gs.kc = 1;
  // the epilogue runs on LDS-staged 64 x 8 tiles where they fit, one plane
  // per block (measured at 256^3: 485 us against 525 us for one-row tiles;
  // marching more planes gains nothing)
  P->ge = G;
  P->ge.kc = 1;
  // the interface terms march up to 64 planes per block (the four-plane
  // prologue of a block, C of planes k-1 .. k+2, is then a small share of its
  // loads), fewer where the grid would give under two blocks per compute unit
  // (measured at 256^3: 8 planes 0.27 ms, 64 planes 0.19 ms)
  P->gi = G;
  {
    const int tx = P->g.txp < 64 ? P->g.txp : 64, ty = vp::kInterfaceThreads / tx;
    const long tiles = (long)(nx / tx) * ((ny + ty - 1) / ty);
    int kc = 64;
    while (kc > 8 && tiles * ((nz + kc - 1) / kc) < 512) kc /= 2;
    P->gi.kc = kc < nz ? kc : nz;
  }
  // geometry of the mixed chain's x passes (the iterates are set per solve)
  vp::ResidualArgs& R = P->rgeo;
  R.mean = nullptr;
  R.dzf = P->dzf;
  R.dzc = P->dzc;
  R.idx2 = 1.0 / (P->dx * P->dx);
  R.idy2 = 1.0 / (P->dy * P->dy);
  R.ny = ny;
  R.nz = nz;
  R.perx = P->bc[0] == vp::BC_P;
  R.pery = P->bc[1] == vp::BC_P;
  R.perz = zper;
  R.outflow = G.outflow;
  return VP_OK;
}

// FP64 chain over nb fields: rhs[b] -> sol[b] (sol[b] may alias rhs[b]);
// the spectra live in nb consecutive slots of N values from `work` (the
// plan's workspace unless a caller passes another buffer)
int solve_f64(poisson_plan* P, int nb, const double* const* rhs, double* const* sol,
              hipStream_t st, double* work = nullptr) {
  const long nrows = (long)P->ny * P->nz, N = P->npts();
  double* w = work ? work : P->work64;
  const vp::Batch<const double> in = vp::batch_of(rhs, nb);
  const vp::Batch<double> out = vp::batch_of(sol, nb);
  VP_LAUNCH(P, K_XFWD, vp::launch_xfwd_f64(in, nb, w, N, P->nx, P->bc[0], nrows, P->tabx64, P->x_pt, st), "x forward", st);
  VP_LAUNCH(P, K_YFWD, vp::launch_y_f64(w, P->nx, P->ny, P->nz * nb, P->bc[1], true, P->taby64, P->y_pt, P->y_lines, st), "y forward", st);
  if (P->z_spec)
    VP_LAUNCH(P, K_Z, vp::launch_zspec_f64(w, P->zs, P->tabz64, P->z_pt, nb, st), "z spectral", st);
  else
    VP_LAUNCH(P, K_Z, vp::launch_zsolve_f64(w, P->z, nb, st), "z solve", st);
  VP_LAUNCH(P, K_YINV, vp::launch_y_f64(w, P->nx, P->ny, P->nz * nb, P->bc[1], false, P->taby64, P->y_pt, P->y_lines, st), "y inverse", st);
  VP_LAUNCH(P, K_XINV, vp::launch_xinv_f64(w, N, out, nb, P->nx, P->bc[0], nrows, P->tabx64, P->x_pt, st), "x inverse", st);
  return VP_OK;
}

// FP32 chain (FP32 spectra, FP64 arithmetic) on FP64 inputs: with iter null
// the x forward reads rhs[b]; otherwise it reads the defect
// rhs[b] - fm[b] - L_h iter[b] (fm may be null: no shift).  out[b] = result,
// or with accum out[b] += result - asub[b] (asub may be null).  o.skip and
// o.norms as in vp::PassOpts.
int solve_f32(poisson_plan* P, int nb, const double* const* rhs, const double* const* iter,
              const double* fm, double* const* out, bool accum, const double* asub,
              vp::PassOpts o, hipStream_t st) {
  const long nrows = (long)P->ny * P->nz, N = P->npts();
  float* w = P->work32;
  const vp::Batch<const double> in = vp::batch_of(rhs, nb);
  const vp::Batch<double> ob = vp::batch_of(out, nb);
  vp::ResidualArgs geo = P->rgeo;
  if (iter) {
    geo.p = vp::batch_of(iter, nb);
    geo.mean = fm;
  }
  vp::ZArgs z = P->z;
  z.skip = o.skip;
  o.nzm = P->nz;
  o.geo = &geo;
  vp::PassOpts fo = o, io = o;
  fo.residual = iter != nullptr;
  fo.sub = nullptr;
  io.sub = asub;
  vp::PassOpts mo = o;  // y passes: flags and tile width only
  mo.sub = nullptr;
  mo.norms = nullptr;
  mo.geo = nullptr;
  mo.lines = P->y_lines;
  if (iter)
    VP_LAUNCH(P, K_RESIDUAL, vp::launch_xfwd_f32(in, nb, w, N, P->nx, P->bc[0], nrows, P->tabx64, P->x_pt, fo, st),
              "x forward residual f32", st);
  else
    VP_LAUNCH(P, K_XFWD32, vp::launch_xfwd_f32(in, nb, w, N, P->nx, P->bc[0], nrows, P->tabx64, P->x_pt, fo, st),
              "x forward f32", st);
  VP_LAUNCH(P, K_YFWD32, vp::launch_y_f32(w, P->nx, P->ny, P->nz * nb, P->bc[1], true, P->taby64, P->y_pt, mo, st), "y forward f32", st);
  if (P->z_spec)
    VP_LAUNCH(P, K_Z32, vp::launch_zspec_f32(w, P->zs, P->tabz64, P->z_pt, nb, o.skip, st),
              "z spectral f32", st);
  else
    VP_LAUNCH(P, K_Z32, vp::launch_zsolve_f32(w, z, nb, st), "z solve f32", st);
  VP_LAUNCH(P, K_YINV32, vp::launch_y_f32(w, P->nx, P->ny, P->nz * nb, P->bc[1], false, P->taby64, P->y_pt, mo, st), "y inverse f32", st);
  VP_LAUNCH(P, K_XINV32, vp::launch_xinv_f32(w, N, ob, nb, P->nx, P->bc[0], nrows, accum, P->tabx64, P->x_pt, io, st),
            "x inverse f32", st);
  return VP_OK;
}

// Mixed precision: p_0 = S32(f), then up to dc_steps times
//   e = S32(f - m - L_h p),  p <- p + e - mean_W(p),
// with m = mean_W(f), removed in FP64 before any FP32 store (a right-hand
// side with a non-zero mean would otherwise leave a defect dominated by it,
// whose FP32 copy loses the part the correction needs); the FP32 chain cannot
// see the constant mode, so the FP64 weighted mean of p is removed by each
// correction instead.  With an outflow end there is no null mode and neither
// mean is removed.  The defect is formed inside the x forward pass of the
// correction (FP64 reads of f and p, FP32 store of its x spectrum); the
// weighted sums behind both means and the norms of the error estimate come
// from the x passes' per-block partial sums, reduced by the control kernel
// after each solve.
// Stopping, per member and on the device: after each correction the error
// left by its FP32 solve is estimated from |defect|, |e| and |p| (see
// k_dc_update) and once that is at most dc_tol the member's flag is set and
// its later passes return at once (no host synchronisation).
// Batch member b keeps f in place, or in work64 slot b when an output
// overwrites it.
int solve_mixed(poisson_plan* P, int nb, const double* const* rhs, double* const* sol,
                hipStream_t st) {
  const long N = P->npts(), nrows = (long)P->ny * P->nz;
  const double* f[vp::kMaxBatch];
  for (int b = 0; b < nb; ++b) {
    f[b] = rhs[b];
    bool clobbered = false;
    for (int c = 0; c < nb; ++c) clobbered = clobbered || sol[c] == rhs[b];
    if (clobbered) {
      VP_HIP(hipMemcpyAsync(P->work64 + b * N, rhs[b], sizeof(double) * N, hipMemcpyDeviceToDevice, st),
             "copy rhs");
      f[b] = P->work64 + b * N;
    }
  }
  double* const pmeans = P->mean + vp::kMaxBatch;      // FP64 weighted mean of p per member
  double* const fmeans = P->mean + 2 * vp::kMaxBatch;  // and of f
  const long nblk = vp::xpass_blocks(P->nx, P->bc[0], P->x_pt, nrows);
  if (nblk < 1 || vp::kNormSlots * nblk > nrows) {
    g_last_error = "mixed solve: x-pass partial sums exceed their buffer";
    return VP_EINVAL;
  }
  const double denom = (double)P->nx * (double)P->ny * P->dz_sum;
  // the first solve reads no flag; the control kernel of step 0 clears them
  vp::PassOpts o;
  o.norms = P->dc_norms;
  int s = solve_f32(P, nb, f, nullptr, nullptr, sol, false, nullptr, o, st);
  if (s) return s;
  VP_HIP(vp::launch_dc_update(P->dc_norms, nblk, nb, 0, P->dc_tol, P->noise_gain, denom,
                              P->dc_state, P->dc_flags, pmeans, fmeans, st),
         "dc update");
  o.skip = P->dc_flags;
  const double* const fm = P->singular ? fmeans : nullptr;
  const double* const asub = P->singular ? pmeans : nullptr;
  for (int it = 1; it <= P->dc_steps; ++it) {
    s = solve_f32(P, nb, f, sol, fm, sol, true, asub, o, st);
    if (s) return s;
    VP_HIP(vp::launch_dc_update(P->dc_norms, nblk, nb, it, P->dc_tol, P->noise_gain, denom,
                                P->dc_state, P->dc_flags, pmeans, fmeans, st),
           "dc update");
  }
  return VP_OK;
}

int solve_any(poisson_plan* P, int nb, const double* const* rhs, double* const* sol,
              hipStream_t st) {
  if (P->precision == VP_PRECISION_MIXED) return solve_mixed(P, nb, rhs, sol, st);
  return solve_f64(P, nb, rhs, sol, st);
}

int solve_one(poisson_plan* P, const double* rhs, double* sol, hipStream_t st) {
  return solve_any(P, 1, &rhs, &sol, st);
}

}  // namespace

extern "C" {

poisson_plan* poisson_plan_create(int nx, int ny, int nz, double dx, double dy, const double* dz,
                                  const char* bc, int precision, int max_batch, int* status) {
  auto fail = [&](int s) -> poisson_plan* {
    if (status) *status = s;
    return nullptr;
  };
  const int chk = poisson_plan_check(nx, ny, nz, dx, dy, dz, bc, precision, max_batch);
  if (chk != VP_OK) return fail(chk);
  char ends[6];
  (void)vp::parse_ends(bc, ends);  // checked above
  int bcs[3];
  for (int d = 0; d < 3; ++d) bcs[d] = vp::direction_code(ends[2 * d], ends[2 * d + 1]);

  poisson_plan* P = new (std::nothrow) poisson_plan();
  if (!P) return fail(VP_ENOMEM);
  P->nx = nx; P->ny = ny; P->nz = nz;
  P->dx = dx; P->dy = dy;
  P->bc[0] = bcs[0]; P->bc[1] = bcs[1]; P->bc[2] = bcs[2];
  std::memcpy(P->ends, ends, 6);
  P->singular = true;
  for (int e = 0; e < 6; ++e) P->singular = P->singular && ends[e] != 'D';
  P->precision = precision;
  P->max_batch = max_batch;
  P->dc_steps = precision == VP_PRECISION_MIXED ? 3 : 0;
  if (hipGetDevice(&P->device) != hipSuccess) {
    delete P;
    return fail(VP_EHIP);
  }
  // set-up of poisson_solve_noalloc on this device (the plan's device is the
  // current one): its static spectrum slot's address, once per device
  if (precision == VP_PRECISION_FP64 && P->npts() <= VP_NOALLOC_MAX_POINTS &&
      !scratch_on(P->device)) {
    delete P;
    return fail(VP_EHIP);
  }
  const int st = plan_init(P, dz);
  if (st != VP_OK) {
    P->release();
    delete P;
    return fail(st);
  }
  if (status) *status = VP_OK;
  return P;
}

void poisson_plan_destroy(poisson_plan* P) {
  if (!P) return;
  (void)hipDeviceSynchronize();
  P->release();
  delete P;
}

int poisson_solve(poisson_plan* P, const double* rhs, double* sol, void* stream) {
  if (!P || !rhs || !sol) return VP_EINVAL;
  return solve_one(P, rhs, sol, static_cast<hipStream_t>(stream));
}

int poisson_solve_batched(poisson_plan* P, int n, const double* const* rhs, double* const* sol,
                          void* stream) {
  if (!P || !rhs || !sol || n < 0 || n > P->max_batch) return VP_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!rhs[i] || !sol[i]) return VP_EINVAL;
  if (n == 0) return VP_OK;
  return solve_any(P, n, rhs, sol, static_cast<hipStream_t>(stream));
}

int poisson_solve_noalloc(poisson_plan* P, const double* rhs, double* sol, void* stream) {
  if (!P || !rhs || !sol) return VP_EINVAL;
  if (P->precision != VP_PRECISION_FP64 || P->npts() > VP_NOALLOC_MAX_POINTS)
    return VP_EUNSUPPORTED;
  int dev = -1;
  VP_HIP(hipGetDevice(&dev), "noalloc device");
  if (dev != P->device) return VP_EINVAL;
  double* w = scratch_on(dev);
  if (!w) return VP_EHIP;
  // no profiling brackets here: they may create events
  const unsigned prof = P->profiling;
  P->profiling = 0;
  const int s = solve_f64(P, 1, &rhs, &sol, static_cast<hipStream_t>(stream), w);
  P->profiling = prof;
  return s;
}

namespace {
// The face stencils hold one face per cell and direction (the upper one): an
// outflow face at a lower end, whose velocity is free, lives in a plane of
// its own (vp_lower_faces), which only the _lf entry points take.
bool lower_out(const poisson_plan* P, int d) { return P->ends[2 * d] == 'D'; }
bool faces_stored(const poisson_plan* P) {
  return !lower_out(P, 0) && !lower_out(P, 1) && !lower_out(P, 2);
}
double* lf_plane(const vp_lower_faces* lf, int d) {
  return lf ? (d == 0 ? lf->u : (d == 1 ? lf->v : lf->w)) : nullptr;
}
// an input / in-out set: a plane exactly for the lower outflow ends
bool lower_in_ok(const poisson_plan* P, const vp_lower_faces* lf) {
  for (int d = 0; d < 3; ++d)
    if (lower_out(P, d) != (lf_plane(lf, d) != nullptr)) return false;
  return true;
}
// an output set: planes only at lower outflow ends (null: not written)
bool lower_out_ok(const poisson_plan* P, const vp_lower_faces* lf) {
  for (int d = 0; d < 3; ++d)
    if (!lower_out(P, d) && lf_plane(lf, d)) return false;
  return true;
}

int project_impl(poisson_plan* P, double* u, double* v, double* w, const vp_lower_faces* lf,
                 const double* phat, const double* rho, double rho0, const double* src, double dt,
                 double* p, hipStream_t st) {
  double* b = P->work64;
  VP_LAUNCH(P, K_RHS, vp::launch_rhs(P->g, u, v, w, phat, rho, rho0, src, dt, b, st), "rhs assembly", st);
  for (int d = 0; d < 3; ++d)
    if (lower_out(P, d))
      VP_LAUNCH(P, K_RHS,
                vp::launch_lower_faces(P->g, vp::LF_RHS, d, lf_plane(lf, d), nullptr, b, nullptr,
                                       phat, rho, rho0, dt, nullptr, st),
                "rhs lower faces", st);
  int s = solve_one(P, b, p, st);
  if (s) return s;
  VP_LAUNCH(P, K_CORRECT, vp::launch_correct(P->gs, u, v, w, p, phat, rho, rho0, dt, st), "correction", st);
  for (int d = 0; d < 3; ++d)
    if (lower_out(P, d))
      VP_LAUNCH(P, K_CORRECT,
                vp::launch_lower_faces(P->g, vp::LF_CORRECT, d, lf_plane(lf, d), nullptr, nullptr, p,
                                       phat, rho, rho0, dt, nullptr, st),
                "correction lower faces", st);
  return VP_OK;
}

int check_extend(const vp_extend_fields& a) {
  if (!a.u || !a.v || !a.w || !a.src || !a.ue || !a.ve || !a.we) return VP_EINVAL;
  const bool hq = a.qx && a.qy && a.qz, hg = a.ug && a.vg && a.wg;
  if ((a.qx || a.qy || a.qz) && !hq) return VP_EINVAL;
  if ((a.ug || a.vg || a.wg) && !hg) return VP_EINVAL;
  if (hq != hg) return VP_EINVAL;
  return VP_OK;
}

// n extensions; with n == 1, lin / lout are the member's lower-face planes
// (u in, u_1^e out) at lower outflow ends
int extend_impl(poisson_plan* P, int n, const vp_extend_fields* a, const vp_lower_faces* lin,
                const vp_lower_faces* lout, hipStream_t st) {
  const long N = P->npts();
  const double* rhs[vp::kMaxBatch];
  double* phi[vp::kMaxBatch];
  for (int b = 0; b < n; ++b) {
    if (check_extend(a[b])) return VP_EINVAL;
    rhs[b] = a[b].src;
    phi[b] = a[b].phi;
    if (!phi[b]) {
      if (P->precision == VP_PRECISION_MIXED) return VP_EINVAL;  // needs a caller buffer
      phi[b] = P->work64 + b * N;  // the x pass writes its own slot in place
    }
  }
  if (n == 0) return VP_OK;
  int s = solve_any(P, n, rhs, phi, st);
  if (s) return s;
  for (int b = 0; b < n; ++b)
    VP_LAUNCH(P, K_EXTEND,
              vp::launch_extend(P->gs, a[b].u, a[b].v, a[b].w, phi[b], a[b].qx, a[b].qy, a[b].qz,
                                a[b].ue, a[b].ve, a[b].we, a[b].ug, a[b].vg, a[b].wg, st),
              "extension", st);
  for (int d = 0; d < 3; ++d)
    if (lower_out(P, d) && lf_plane(lout, d))
      VP_LAUNCH(P, K_EXTEND,
                vp::launch_lower_faces(P->g, vp::LF_EXTEND, d, lf_plane(lin, d), lf_plane(lout, d),
                                       nullptr, nullptr, nullptr, nullptr, 1.0, 1.0, phi[0], st),
                "extension lower faces", st);
  return VP_OK;
}

int step_impl(poisson_plan* P, double* u, double* v, double* w, const vp_lower_faces* lf,
              const double* phat, const double* rho, double rho0, const double* src_p, double dt,
              double* p, const double* src_ext, const double* qx, const double* qy,
              const double* qz, double* ue, double* ve, double* we, const vp_lower_faces* lfe,
              double* ug, double* vg, double* wg, double* phi, hipStream_t st) {
  double* b = P->work64;
  VP_LAUNCH(P, K_RHS, vp::launch_rhs(P->g, u, v, w, phat, rho, rho0, src_p, dt, b, st),
            "rhs assembly", st);
  for (int d = 0; d < 3; ++d)
    if (lower_out(P, d))
      VP_LAUNCH(P, K_RHS,
                vp::launch_lower_faces(P->g, vp::LF_RHS, d, lf_plane(lf, d), nullptr, b, nullptr,
                                       phat, rho, rho0, dt, nullptr, st),
                "rhs lower faces", st);
  // the Stefan potential does not depend on the pressure: with room for two
  // fields both solves run as one batch (one launch per pass, the same bits)
  int s;
  if (P->max_batch >= 2) {
    const double* rhs2[2] = {b, src_ext};
    double* sol2[2] = {p, phi};
    s = solve_any(P, 2, rhs2, sol2, st);
  } else {
    s = solve_one(P, b, p, st);
    if (!s) s = solve_one(P, src_ext, phi, st);
  }
  if (s) return s;
  VP_LAUNCH(P, K_EPILOGUE,
            vp::launch_step_epilogue(P->ge, u, v, w, p, phat, rho, rho0, dt, phi, qx, qy, qz, ue,
                                     ve, we, ug, vg, wg, st),
            "step epilogue", st);
  for (int d = 0; d < 3; ++d)
    if (lower_out(P, d))
      VP_LAUNCH(P, K_EPILOGUE,
                vp::launch_lower_faces(P->g, vp::LF_STEP, d, lf_plane(lf, d), lf_plane(lfe, d),
                                       nullptr, p, phat, rho, rho0, dt, phi, st),
                "step lower faces", st);
  return VP_OK;
}

int check_step(double* u, double* v, double* w, const double* phat, const double* rho,
               double rho0, double dt, double* p, const double* src_ext, const double* qx,
               const double* qy, const double* qz, double* ue, double* ve, double* we,
               double* ug, double* vg, double* wg, double* phi) {
  if (!u || !v || !w || !phat || !rho || !p || !src_ext || !phi || !(rho0 > 0) || !(dt > 0))
    return VP_EINVAL;
  const bool hq = qx && qy && qz, hg = ug && vg && wg, he = ue && ve && we;
  if ((qx || qy || qz) && !hq) return VP_EINVAL;
  if ((ug || vg || wg) && !hg) return VP_EINVAL;
  if ((ue || ve || we) && !he) return VP_EINVAL;
  if (hq != hg) return VP_EINVAL;
  if (phi == p) return VP_EINVAL;
  return VP_OK;
}
}  // namespace

int project(poisson_plan* P, double* u, double* v, double* w, const double* phat,
            const double* rho, double rho0, const double* src, double dt, double* p,
            void* stream) {
  if (!P || !u || !v || !w || !phat || !rho || !p || !(rho0 > 0) || !(dt > 0)) return VP_EINVAL;
  if (!faces_stored(P)) return VP_EUNSUPPORTED;
  return project_impl(P, u, v, w, nullptr, phat, rho, rho0, src, dt, p,
                      static_cast<hipStream_t>(stream));
}

int project_lf(poisson_plan* P, double* u, double* v, double* w, const vp_lower_faces* lower,
               const double* phat, const double* rho, double rho0, const double* src, double dt,
               double* p, void* stream) {
  if (!P || !u || !v || !w || !phat || !rho || !p || !(rho0 > 0) || !(dt > 0)) return VP_EINVAL;
  if (!lower_in_ok(P, lower)) return VP_EINVAL;
  return project_impl(P, u, v, w, lower, phat, rho, rho0, src, dt, p,
                      static_cast<hipStream_t>(stream));
}

int extend_liquid_velocity_batched(poisson_plan* P, int n, const vp_extend_fields* a,
                                   void* stream) {
  if (!P || !a || n < 0 || n > P->max_batch) return VP_EINVAL;
  if (!faces_stored(P)) return VP_EUNSUPPORTED;
  return extend_impl(P, n, a, nullptr, nullptr, static_cast<hipStream_t>(stream));
}

int extend_liquid_velocity(poisson_plan* P, const double* u, const double* v, const double* w,
                           const double* src, const double* qx, const double* qy,
                           const double* qz, double* ue, double* ve, double* we, double* ug,
                           double* vg, double* wg, double* phi, void* stream) {
  if (!P) return VP_EINVAL;
  const vp_extend_fields a = {u, v, w, src, qx, qy, qz, ue, ve, we, ug, vg, wg, phi};
  return extend_liquid_velocity_batched(P, 1, &a, stream);
}

int extend_liquid_velocity_lf(poisson_plan* P, const double* u, const double* v, const double* w,
                              const vp_lower_faces* lower, const double* src, const double* qx,
                              const double* qy, const double* qz, double* ue, double* ve,
                              double* we, const vp_lower_faces* lower_e, double* ug, double* vg,
                              double* wg, double* phi, void* stream) {
  if (!P || !lower_in_ok(P, lower) || !lower_out_ok(P, lower_e)) return VP_EINVAL;
  const vp_extend_fields a = {u, v, w, src, qx, qy, qz, ue, ve, we, ug, vg, wg, phi};
  return extend_impl(P, 1, &a, lower, lower_e, static_cast<hipStream_t>(stream));
}

int vof_step(poisson_plan* P, double* u, double* v, double* w, const double* phat,
             const double* rho, double rho0, const double* src_p, double dt, double* p,
             const double* src_ext, const double* qx, const double* qy, const double* qz,
             double* ue, double* ve, double* we, double* ug, double* vg, double* wg, double* phi,
             void* stream) {
  if (!P || check_step(u, v, w, phat, rho, rho0, dt, p, src_ext, qx, qy, qz, ue, ve, we, ug, vg,
                       wg, phi))
    return VP_EINVAL;
  if (!faces_stored(P)) return VP_EUNSUPPORTED;
  return step_impl(P, u, v, w, nullptr, phat, rho, rho0, src_p, dt, p, src_ext, qx, qy, qz, ue, ve,
                   we, nullptr, ug, vg, wg, phi, static_cast<hipStream_t>(stream));
}

int vof_step_lf(poisson_plan* P, double* u, double* v, double* w, const vp_lower_faces* lower,
                const double* phat, const double* rho, double rho0, const double* src_p,
                double dt, double* p, const double* src_ext, const double* qx, const double* qy,
                const double* qz, double* ue, double* ve, double* we,
                const vp_lower_faces* lower_e, double* ug, double* vg, double* wg, double* phi,
                void* stream) {
  if (!P || check_step(u, v, w, phat, rho, rho0, dt, p, src_ext, qx, qy, qz, ue, ve, we, ug, vg,
                       wg, phi))
    return VP_EINVAL;
  if (!lower_in_ok(P, lower) || !lower_out_ok(P, lower_e)) return VP_EINVAL;
  return step_impl(P, u, v, w, lower, phat, rho, rho0, src_p, dt, p, src_ext, qx, qy, qz, ue, ve,
                   we, lower_e, ug, vg, wg, phi, static_cast<hipStream_t>(stream));
}

int vof_step_interface(poisson_plan* P, double* u, double* v, double* w, const double* phat,
                       const double* rho, double rho0, const double* C, const double* mdot,
                       double rho1, double rho2, int phase, double dt, double* p, double* s,
                       double* ue, double* ve, double* we, double* ug, double* vg, double* wg,
                       double* phi, void* stream) {
  if (!P || !u || !v || !w || !phat || !rho || !C || !mdot || !p || !s || !phi || !ug || !vg ||
      !wg || !(rho0 > 0) || !(dt > 0) || !(rho1 > 0) || !(rho2 > 0) || (phase != 1 && phase != 2))
    return VP_EINVAL;
  if ((ue || ve || we) && !(ue && ve && we)) return VP_EINVAL;
  if (phi == p || s == p || s == phi) return VP_EINVAL;
  if (!faces_stored(P)) return VP_EUNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* b = P->work64;
  vp::IfStepArgs a;
  a.u = u;
  a.v = v;
  a.w = w;
  a.ph = phat;
  a.rho = rho;
  a.rho0 = rho0;
  a.dt = dt;
  a.b = b;
  VP_LAUNCH(P, K_RHS, vp::launch_rhs_interface(P->gi, C, mdot, rho1, rho2, s, a, st),
            "rhs with interface terms", st);
  int e;
  if (P->max_batch >= 2) {
    const double* rhs2[2] = {b, s};
    double* sol2[2] = {p, phi};
    e = solve_any(P, 2, rhs2, sol2, st);
  } else {
    e = solve_one(P, b, p, st);
    if (!e) e = solve_one(P, s, phi, st);
  }
  if (e) return e;
  vp::IfStepArgs q;
  q.uo = u;
  q.vo = v;
  q.wo = w;
  q.ph = phat;
  q.rho = rho;
  q.rho0 = rho0;
  q.dt = dt;
  q.p = p;
  q.phi = phi;
  q.ue = ue;
  q.ve = ve;
  q.we = we;
  q.ug = ug;
  q.vg = vg;
  q.wg = wg;
  VP_LAUNCH(P, K_EPILOGUE,
            vp::launch_epilogue_interface(P->gi, C, mdot, phase == 1 ? rho1 : rho2, q, st),
            "step epilogue with interface terms", st);
  return VP_OK;
}

int interface_terms(poisson_plan* P, const double* C, const double* mdot, double rho1,
                    double rho2, int phase, double* s, double* qx, double* qy, double* qz,
                    void* stream) {
  if (!P || !C || !mdot || !s || !qx || !qy || !qz || !(rho1 > 0) || !(rho2 > 0) ||
      (phase != 1 && phase != 2))
    return VP_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  VP_LAUNCH(P, K_INTERFACE,
            vp::launch_interface(P->gi, C, mdot, rho1, rho2, phase == 1 ? rho1 : rho2, s, qx,
                                 qy, qz, st),
            "interface terms", st);
  return VP_OK;
}

int vof_advect(poisson_plan* P, const double* C, const double* ug, const double* vg,
               const double* wg, const vp_lower_faces* lower, double dt, double beta,
               int deflation, double* C_new, void* stream) {
  if (!P || !C || !ug || !vg || !wg || !C_new || C_new == C || !(dt > 0) || !(beta > 0) ||
      (deflation != 0 && deflation != 1))
    return VP_EINVAL;
  if (!lower_in_ok(P, lower)) return faces_stored(P) ? VP_EINVAL : VP_EUNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double* lo[3] = {lf_plane(lower, 0), lf_plane(lower, 1), lf_plane(lower, 2)};
  // C** of the y sweep lives in workspace slot 0
  for (int sw = 0; sw < 3; ++sw)
    VP_LAUNCH(P, K_ADV_X + sw,
              vp::launch_advect(P->gs, C, ug, vg, wg, lo, dt, beta, deflation, P->work64, C_new,
                                sw, st),
              "advect sweep", st);
  return VP_OK;
}

int poisson_plan_set_mixed(poisson_plan* P, int dc_steps) {
  if (!P || P->precision != VP_PRECISION_MIXED || dc_steps < 0 || dc_steps > 8) return VP_EINVAL;
  P->dc_steps = dc_steps;
  return VP_OK;
}

int poisson_plan_set_mixed_tol(poisson_plan* P, double tol) {
  if (!P || P->precision != VP_PRECISION_MIXED || !(tol == tol)) return VP_EINVAL;
  P->dc_tol = tol;
  return VP_OK;
}

int poisson_plan_mixed_report(poisson_plan* P, int n, int* steps, double* estimate,
                              void* stream) {
  if (!P || P->precision != VP_PRECISION_MIXED || n < 1 || n > P->max_batch) return VP_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double h[4 * vp::kMaxBatch];
  VP_HIP(hipMemcpyAsync(h, P->dc_state, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, st),
         "dc report");
  VP_HIP(hipStreamSynchronize(st), "dc report sync");
  for (int b = 0; b < n; ++b) {
    if (steps) steps[b] = (int)h[4 * b + 2];
    if (estimate) estimate[b] = h[4 * b + 1];
  }
  return VP_OK;
}

int poisson_plan_last_mean(poisson_plan* P, double* mean_out, void* stream) {
  if (!P || !mean_out) return VP_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  VP_HIP(hipMemcpyAsync(mean_out, P->mean, sizeof(double), hipMemcpyDeviceToHost, st), "mean");
  VP_HIP(hipStreamSynchronize(st), "mean sync");
  return VP_OK;
}

long long poisson_plan_device_bytes(const poisson_plan* P) { return P ? P->bytes : -1; }

const char* poisson_strerror(int status) {
  switch (status) {
    case VP_OK: return "ok";
    case VP_EINVAL: return "invalid argument";
    case VP_EUNSUPPORTED: return "unsupported size or boundary condition";
    case VP_ENOMEM: return "device out of memory";
    case VP_EHIP: return g_last_error.empty() ? "HIP runtime error" : g_last_error.c_str();
    default: return "unknown status";
  }
}

int poisson_plan_tune(poisson_plan* P, const char* key, int value) {
  if (!P || !key) return VP_EINVAL;
  const std::string k(key);
  if (k == "z_lines") {
    if (value != 8 && value != 16 && value != 32) return VP_EINVAL;
    P->z.lines = value;
    return VP_OK;
  }
  if (k == "x_radix" || k == "y_radix") {
    if (value != 8 && value != 16) return VP_EINVAL;
    (k == "x_radix" ? P->x_pt : P->y_pt) = value;
    return VP_OK;
  }
  if (k == "z_spectral") {
    if (value != 0 && value != 1) return VP_EINVAL;
    if (value == 1 && !P->z_spec_ok) return VP_EUNSUPPORTED;
    P->z_spec = value;
    return VP_OK;
  }
  if (k == "z_radix") {
    if (value != 8 && value != 16) return VP_EINVAL;
    P->z_pt = value;
    return VP_OK;
  }
  if (k == "y_lines") {
    if (value < 0 || value > 256 || (value & (value - 1))) return VP_EINVAL;
    P->y_lines = value;
    return VP_OK;
  }
  if (k == "z_spectral_lines") {
    if (value < 0 || value > 256 || (value & (value - 1))) return VP_EINVAL;
    P->zs.lines = value;
    return VP_OK;
  }
  if (k == "rhs_tiled") {
    if (value != 0 && value != 8 && value != 16) return VP_EINVAL;
    P->g.tiled = value;
    return VP_OK;
  }
  if (k == "epilogue_tiled") {
    if (value != 0 && value != 8 && value != 16) return VP_EINVAL;
    P->ge.tiled = value;
    return VP_OK;
  }
  if (k == "epilogue_planes") {
    if (value < 1 || value > P->nz) return VP_EINVAL;
    P->ge.kc = value;
    return VP_OK;
  }
  if (k == "z_segment") {
    if ((value != 8 && value != 16) || (P->nz + value - 1) / value > 64) return VP_EINVAL;
    set_z_segment(P->z, value);
    return VP_OK;
  }
  if (k == "interface_planes") {
    if (value < 1 || value > P->nz) return VP_EINVAL;
    P->gi.kc = value;
    return VP_OK;
  }
  if (k == "interface_tile") {
    if (value < 8 || value > 64 || (value & (value - 1)) || value > P->g.txp) return VP_EINVAL;
    P->gi.txp = value;  // the tile width is min(txp, 64)
    return VP_OK;
  }
  if (k == "stream_planes") {
    if (value < 1 || value > P->nz) return VP_EINVAL;
    P->gs.kc = value;
    return VP_OK;
  }
  if (k == "stream_tiled") {
    if (value != 0 && value != 8 && value != 16) return VP_EINVAL;
    P->gs.tiled = value;
    return VP_OK;
  }
  if (k == "stencil_planes") {
    if (value < 1 || value > P->nz) return VP_EINVAL;
    P->g.kc = value;
    return VP_OK;
  }
  return VP_EINVAL;
}

}  // extern "C"

namespace {

// median time in ms of `reps` runs of launch(), after one untimed run
template <typename F>
int time_ms(hipStream_t st, int reps, F launch, float* out) {
  int s = launch();
  if (s) return s;
  std::vector<float> t;
  hipEvent_t a = nullptr, b = nullptr;
  VP_HIP(hipEventCreate(&a), "tune event");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return hip_fail(hipErrorOutOfMemory, "tune event");
  }
  for (int r = 0; r < reps && s == VP_OK; ++r) {
    (void)hipEventRecord(a, st);
    s = launch();
    (void)hipEventRecord(b, st);
    float ms = 0.f;
    if (s == VP_OK && hipEventSynchronize(b) == hipSuccess &&
        hipEventElapsedTime(&ms, a, b) == hipSuccess)
      t.push_back(ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (s) return s;
  if (t.empty()) return hip_fail(hipErrorUnknown, "tune timing");
  std::sort(t.begin(), t.end());
  *out = t[t.size() / 2];
  return VP_OK;
}

// pick the candidate of `knob` (an int of the plan) with the smallest median
// time of `launch`; the knob is left at the winner
template <typename F>
int pick(hipStream_t st, int* knob, const std::vector<int>& cands, F launch, int* chosen) {
  float best = 0.f;
  int arg = *knob;
  for (size_t i = 0; i < cands.size(); ++i) {
    *knob = cands[i];
    float ms = 0.f;
    const int s = time_ms(st, 5, launch, &ms);
    if (s) return s;
    if (i == 0 || ms < best) {
      best = ms;
      arg = cands[i];
    }
  }
  *knob = arg;
  if (chosen) *chosen = arg;
  return VP_OK;
}

}  // namespace

extern "C" {

int poisson_plan_autotune(poisson_plan* P, int nb, void* stream, int* chosen) {
  if (!P || nb < 1 || nb > P->max_batch) return VP_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long N = P->npts(), nrows = (long)P->ny * P->nz;
  const bool mixed = P->precision == VP_PRECISION_MIXED;
  // the passes run in place on the zeroed workspace (each block owns the
  // rows or columns it rewrites); the result is discarded
  VP_HIP(hipMemsetAsync(P->work64, 0, sizeof(double) * N * P->max_batch, st), "tune clear");
  if (mixed) VP_HIP(hipMemsetAsync(P->work32, 0, sizeof(float) * N * P->max_batch, st), "tune clear");
  const double* in64[vp::kMaxBatch];
  double* out64[vp::kMaxBatch];
  for (int b = 0; b < nb; ++b) {
    in64[b] = P->work64 + b * N;
    out64[b] = P->work64 + b * N;
  }
  const vp::Batch<const double> bin = vp::batch_of(in64, nb);
  const vp::Batch<double> bout = vp::batch_of(out64, nb);
  int res[8] = {P->x_pt, P->y_pt, P->z.lines, P->g.kc, P->z_spec, P->z_pt, P->y_lines, P->zs.lines};
  int s;
  auto hs = [](hipError_t e) { return e == hipSuccess ? VP_OK : hip_fail(e, "tune launch"); };
  // x passes: forward + inverse
  s = pick(st, &P->x_pt, {16, 8}, [&]() -> int {
    if (mixed) {
      // the x passes of a correction step: residual forward, accumulating
      // inverse, both with their partial sums
      vp::ResidualArgs geo = P->rgeo;
      geo.p = bin;
      vp::PassOpts o{};
      o.geo = &geo;
      o.norms = P->dc_norms;
      o.residual = true;
      int e = hs(vp::launch_xfwd_f32(bin, nb, P->work32, N, P->nx, P->bc[0], nrows, P->tabx64,
                                     P->x_pt, o, st));
      if (e) return e;
      o.residual = false;
      return hs(vp::launch_xinv_f32(P->work32, N, bout, nb, P->nx, P->bc[0], nrows, true,
                                    P->tabx64, P->x_pt, o, st));
    }
    int e = hs(vp::launch_xfwd_f64(bin, nb, P->work64, N, P->nx, P->bc[0], nrows, P->tabx64,
                                   P->x_pt, st));
    if (e) return e;
    return hs(vp::launch_xinv_f64(P->work64, N, bout, nb, P->nx, P->bc[0], nrows, P->tabx64,
                                  P->x_pt, st));
  }, &res[0]);
  if (s) return s;
  // y passes: forward + inverse, radix then tile width
  auto ypair = [&]() -> int {
    vp::PassOpts yo{};
    yo.lines = P->y_lines;
    for (int fwd = 1; fwd >= 0; --fwd) {
      const int e = mixed ? hs(vp::launch_y_f32(P->work32, P->nx, P->ny, P->nz * nb, P->bc[1],
                                                fwd != 0, P->taby64, P->y_pt, yo, st))
                          : hs(vp::launch_y_f64(P->work64, P->nx, P->ny, P->nz * nb, P->bc[1],
                                                fwd != 0, P->taby64, P->y_pt, P->y_lines, st));
      if (e) return e;
    }
    return VP_OK;
  };
  s = pick(st, &P->y_pt, {16, 8}, ypair, &res[1]);
  if (s) return s;
  s = pick(st, &P->y_lines, {0, 8, 4}, ypair, nullptr);
  if (s) return s;
  // z pass: lines per block of the tridiagonal solve, then (uniform z) the
  // spectral pass's radix against the best tridiagonal time
  if (P->nz > 1) {
    const int spec = P->z_spec;
    P->z_spec = 0;
    auto zpass = [&]() -> int {
      if (P->z_spec)
        return mixed ? hs(vp::launch_zspec_f32(P->work32, P->zs, P->tabz64, P->z_pt, nb, nullptr, st))
                     : hs(vp::launch_zspec_f64(P->work64, P->zs, P->tabz64, P->z_pt, nb, st));
      return mixed ? hs(vp::launch_zsolve_f32(P->work32, P->z, nb, st))
                   : hs(vp::launch_zsolve_f64(P->work64, P->z, nb, st));
    };
    // segment length and lines per block together (at most 64 segments)
    int zcode = P->z.seg * 100 + P->z.lines;
    std::vector<int> zc;
    for (int seg : {16, 8})
      if ((P->nz + seg - 1) / seg <= 64)
        for (int lines : {8, 16, 32}) zc.push_back(seg * 100 + lines);
    auto zapply = [&](int code) {
      set_z_segment(P->z, code / 100);
      P->z.lines = code % 100;
    };
    s = pick(st, &zcode, zc, [&]() -> int {
      zapply(zcode);
      return zpass();
    }, nullptr);
    if (s) return s;
    zapply(zcode);
    res[2] = P->z.lines;
    if (P->z_spec_ok) {
      // codes: 0 = tridiagonal (tuned lines), else spectral: radix * 1000 +
      // column pairs per block (0: default width)
      int mode = 0;
      auto apply = [&](int m) {
        P->z_spec = m != 0;
        if (m) {
          P->z_pt = m / 1000;
          P->zs.lines = m % 1000;
        }
      };
      s = pick(st, &mode, {0, 16000, 16008, 16004, 8000, 8008, 8004}, [&]() -> int {
        apply(mode);
        return zpass();
      }, nullptr);
      if (s) return s;
      apply(mode);
    } else {
      P->z_spec = spec;
    }
  }
  // marching stencils: planes per block of the right-hand-side kernel, when
  // the workspace has a second field to write to
  double* second = P->max_batch > 1 ? P->work64 + N : nullptr;
  if (second) {
    std::vector<int> cands;
    for (int kc : {1, 2, 4, 8, 16, 32, vp::stencil_default_planes(P->nx, P->ny, P->nz)}) {
      vp::GridArgs g = P->g;
      g.kc = kc;
      if (kc <= P->nz && std::find(cands.begin(), cands.end(), kc) == cands.end())
        cands.push_back(kc);
    }
    const double* f = P->work64;
    s = pick(st, &P->g.kc, cands, [&]() -> int {
      return hs(vp::launch_rhs(P->g, f, f, f, f, f, 1.0, f, 1.0, second, st));
    }, &res[3]);
    if (s) return s;
  }
  res[4] = P->z_spec;
  res[5] = P->z_pt;
  res[6] = P->y_lines;
  res[7] = P->zs.lines;
  if (chosen)
    for (int i = 0; i < 8; ++i) chosen[i] = res[i];
  return VP_OK;
}

int poisson_plan_get_tuning(poisson_plan* P, const char* key, int* value) {
  if (!P || !key || !value) return VP_EINVAL;
  const std::string k(key);
  if (k == "x_radix") *value = P->x_pt;
  else if (k == "y_radix") *value = P->y_pt;
  else if (k == "z_lines") *value = P->z.lines;
  else if (k == "stencil_planes") *value = P->g.kc;
  else if (k == "stream_planes") *value = P->gs.kc;
  else if (k == "stream_tiled") *value = P->gs.tiled;
  else if (k == "rhs_tiled") *value = P->g.tiled;
  else if (k == "z_spectral") *value = P->z_spec;
  else if (k == "z_radix") *value = P->z_pt;
  else if (k == "z_spectral_lines") *value = P->zs.lines;
  else if (k == "y_lines") *value = P->y_lines;
  else if (k == "epilogue_tiled") *value = P->ge.tiled;
  else if (k == "epilogue_planes") *value = P->ge.kc;
  else if (k == "interface_planes") *value = P->gi.kc;
  else if (k == "interface_tile") *value = P->gi.txp < 64 ? P->gi.txp : 64;
  else if (k == "z_segment") *value = P->z.seg;
  else return VP_EINVAL;
  return VP_OK;
}

int poisson_plan_set_profiling(poisson_plan* P, int class_mask) {
  if (!P) return VP_EINVAL;
  P->profiling = (unsigned)class_mask;
  return VP_OK;
}

int poisson_plan_kernel_times(poisson_plan* P, double* total_ms, int* launches, int n) {
  if (!P || n < 0 || (n > 0 && (!total_ms || !launches))) return VP_EINVAL;
  for (int i = 0; i < n; ++i) {
    total_ms[i] = 0.0;
    launches[i] = 0;
  }
  int status = VP_OK;
  for (auto& m : P->marks) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(m.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.a, m.b);
    if (e != hipSuccess && status == VP_OK) status = hip_fail(e, "kernel timing");
    if (m.cls < n) {
      total_ms[m.cls] += ms;
      launches[m.cls] += 1;
    }
    P->pool.push_back(m.a);
    P->pool.push_back(m.b);
  }
  P->marks.clear();
  return status;
}

const char* poisson_kernel_class_name(int cls) {
  return (cls >= 0 && cls < K_NCLASS) ? kClassNames[cls] : nullptr;
}

const char* vofpoisson_version(void) { return "vofpoisson 0.1 (gfx950)"; }

}  // extern "C"
