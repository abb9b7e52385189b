// y passes of the spectral Poisson solve: every y-line (columns of a
// z-plane), tiles of consecutive columns so that every row access of a
// wavefront is contiguous.
#include "transform_passes.hpp"

namespace vp {

// ---------------------------------------------------------------------------
// y kernels: block (tile, plane); tile = 2*lines columns x N rows; thread
// (q, t) with q fastest, so a wavefront reads 2*lines consecutive columns.
// Blocks take the planes (of every batch member) in reverse: the pass before
// (x forward, z) wrote the last planes last, so they are the likeliest to
// still sit in the Infinity Cache when the y pass starts (measured at 256^3,
// two fields per launch: y forward 100 -> 91 us).
// T: arithmetic and LDS type; TS: type of the data in HBM (float in the mixed
// chain, which computes in FP64 and rounds only what it stores).
// ---------------------------------------------------------------------------
template <typename T, typename TS, int N, int BC, int PTM>
__global__ __launch_bounds__(PTM == 8 ? 512 : 256) void k_yfwd(TS* __restrict__ data, int nx,
                                                               long plane, int llines,
                                                               const T* __restrict__ tab,
                                                               int nzm,
                                                               const int* __restrict__ skip) {
  using T2 = typename Vec2<T>::type;
  using S2 = typename Vec2<TS>::type;
  extern __shared__ unsigned char smem_raw[];
  const uint2 tl = xcd_layer(blockIdx.x, blockIdx.y, gridDim.x, gridDim.y);
  const int by = gridDim.y - 1 - tl.y;  // plane, last first
  if (skip && skip[by / nzm]) return;  // member already converged (whole block)
  const int lines = 1 << llines;
  const int q = threadIdx.x & (lines - 1), t = threadIdx.x >> llines;
  S2* col = reinterpret_cast<S2*>(data + (long)by * plane + (long)tl.x * 2 * lines + 2 * q);
  const int nx2 = nx >> 1;  // row stride in S2 units
  YLds<T, N> lds(reinterpret_cast<T2*>(smem_raw), q, lines);
  forward_body<T, N, BC, PTM>(
      lds, t, tab,
      [&](int e, T& r, T& i) {
        const S2 v = col[(long)e * nx2];
        r = T(v.x);
        i = T(v.y);
      },
      [&](int c0, T a0, T b0, int c1, T a1, T b1) {
        S2 v0, v1;
        v0.x = TS(a0);
        v0.y = TS(b0);
        v1.x = TS(a1);
        v1.y = TS(b1);
        col[(long)c0 * nx2] = v0;
        col[(long)c1 * nx2] = v1;
      });
}

template <typename T, typename TS, int N, int BC, int PTM>
__global__ __launch_bounds__(PTM == 8 ? 512 : 256) void k_yinv(TS* __restrict__ data, int nx,
                                                               long plane, int llines,
                                                               const T* __restrict__ tab,
                                                               int nzm,
                                                               const int* __restrict__ skip) {
  using T2 = typename Vec2<T>::type;
  using S2 = typename Vec2<TS>::type;
  extern __shared__ unsigned char smem_raw[];
  const uint2 tl = xcd_layer(blockIdx.x, blockIdx.y, gridDim.x, gridDim.y);
  const int by = gridDim.y - 1 - tl.y;  // plane, last first
  if (skip && skip[by / nzm]) return;  // member already converged (whole block)
  const int lines = 1 << llines;
  const int q = threadIdx.x & (lines - 1), t = threadIdx.x >> llines;
  S2* col = reinterpret_cast<S2*>(data + (long)by * plane + (long)tl.x * 2 * lines + 2 * q);
  const int nx2 = nx >> 1;
  YLds<T, N> lds(reinterpret_cast<T2*>(smem_raw), q, lines);
  inverse_body<T, N, BC, PTM>(
      lds, t, tab,
      [&](int c0, int c1, T& a0, T& b0, T& a1, T& b1) {
        const S2 v0 = col[(long)c0 * nx2], v1 = col[(long)c1 * nx2];
        a0 = T(v0.x);
        b0 = T(v0.y);
        a1 = T(v1.x);
        b1 = T(v1.y);
      },
      [&](int e, T r, T i) {
        S2 v;
        v.x = TS(r);
        v.y = TS(i);
        col[(long)e * nx2] = v;
      });
}

template <typename T, typename TS, int N, int BC, bool INV, int PTM>
__global__ __launch_bounds__(512) void k_yq(TS* __restrict__ data, int nx, long plane, int lcols,
                                             const T* __restrict__ tab, int nzm,
                                             const int* __restrict__ skip) {
  using T2 = typename Vec2<T>::type;
  extern __shared__ unsigned char smem_raw[];
  const uint2 tl = xcd_layer(blockIdx.x, blockIdx.y, gridDim.x, gridDim.y);
  const int by = gridDim.y - 1 - tl.y;  // plane, last first
  if (skip && skip[by / nzm]) return;  // member already converged (whole block)
  const int cols = 1 << lcols;
  const int q = threadIdx.x & (cols - 1), t = threadIdx.x >> lcols;
  TS* col = data + (long)by * plane + (long)tl.x * cols + q;
  YLds<T, N / 2> lds(reinterpret_cast<T2*>(smem_raw), q, cols);
  if constexpr (INV) {
    quarter_body<T, N, PTM>(
        lds, t, tab, [&](int c, T& v) { v = T(col[(long)c * nx]); },
        [&](int e, T v) { col[(long)qpos<N, BC>(e) * nx] = TS(T(2) * v); });
  } else {
    quarter_body<T, N, PTM>(
        lds, t, tab, [&](int e, T& v) { v = T(col[(long)qpos<N, BC>(e) * nx]); },
        [&](int c, T v) { col[(long)c * nx] = TS(v); });
  }
}

static int ypass_lines(int nx, int ny) {
  int lines = pass_threads(ny) / fft_tpl(ny);
  if (lines < 1) lines = 1;
  if (lines > pow2_part(nx) / 2) lines = (int)(pow2_part(nx) / 2);  // 2 lines divide nx
  return lines;
}

#if VP_IN_PART(1)
int ypass_tile_cols(int nx, int ny) { return 2 * ypass_lines(nx, ny); }
#endif

// quarter-wave y pass: one column per line, 2*lines columns per block
template <typename T, typename TS, int BC, bool FWD, int PTM>
static hipError_t launch_yq_pt(TS* data, int nx, int ny, int nplanes, const T* tab, int lines,
                               int nzm, const int* skip, hipStream_t st) {
  using T2 = typename Vec2<T>::type;
  const int cols = 2 * lines;
  int lc = 0;
  while ((1 << lc) < cols) ++lc;
  const long plane = (long)nx * ny;
  const dim3 grid((unsigned)(nx / cols), (unsigned)nplanes);
#define VP_YQ(NN)                                                                  \
  case NN: {                                                                       \
    const int nthr = cols * FftShape<NN / 2, PTM>::TPL;                            \
    const size_t shm = sizeof(T2) * (size_t)lds_len<NN / 2>() * (cols + 1);        \
    auto kern = &k_yq<T, TS, NN, BC, !FWD, canon_ptm<NN, PTM>()>;                              \
    if (nthr > 512) return hipErrorInvalidValue;                                   \
    if (shm > 65536) {                                                             \
      const hipError_t e = allow_large_lds(kern);                                  \
      if (e != hipSuccess) return e;                                               \
    }                                                                              \
    hipLaunchKernelGGL(kern, grid, dim3(nthr), shm, st, data, nx, plane, lc, tab, nzm, skip); \
    break;                                                                         \
  }
  switch (ny) {
    VP_SIZES(VP_YQ)
    default: return hipErrorInvalidValue;
  }
#undef VP_YQ
  return hipGetLastError();
}

template <typename T, typename TS, int BC, bool FWD, int PTM>
static hipError_t launch_ystd_pt(TS* data, int nx, int ny, int nplanes, const T* tab, int lines,
                                 int nzm, const PassOpts& o, hipStream_t st) {
  using T2 = typename Vec2<T>::type;
  int ll = 0;
  while ((1 << ll) < lines) ++ll;
  const long plane = (long)nx * ny;
  const dim3 grid((unsigned)(nx / (2 * lines)), (unsigned)nplanes);
#define VP_Y(NN)                                                                   \
  case NN: {                                                                       \
    const int nthr = lines * FftShape<NN, PTM>::TPL;                               \
    const size_t shm = sizeof(T2) * (size_t)lds_len<NN>() * (lines + 1);           \
    constexpr int PC = canon_ptm<NN, PTM>();                                               \
    auto kern = FWD ? &k_yfwd<T, TS, NN, BC, PC> : &k_yinv<T, TS, NN, BC, PC>;                     \
    if (shm > 65536) {                                                             \
      const hipError_t e = allow_large_lds(kern);                                  \
      if (e != hipSuccess) return e;                                               \
    }                                                                              \
    hipLaunchKernelGGL(kern, grid, dim3(nthr), shm, st, data, nx, plane, ll, tab, nzm, \
                       o.skip);                                                    \
    break;                                                                         \
  }
  switch (ny) {
    VP_SIZES(VP_Y)
    default: return hipErrorInvalidValue;
  }
#undef VP_Y
  return hipGetLastError();
}

template <typename T, typename TS, int BC, bool FWD, int PTM>
static hipError_t launch_y_pt(TS* data, int nx, int ny, int nplanes, const T* tab,
                              const PassOpts& o, hipStream_t st) {
  int lines = ypass_lines(nx, ny);
  if (o.lines > 0 && o.lines < lines) lines = o.lines;
  const int nzm = o.nzm > 0 ? o.nzm : nplanes;
  if constexpr (BC == BC_ND || BC == BC_DN)
    return launch_yq_pt<T, TS, BC, FWD, PTM>(data, nx, ny, nplanes, tab, lines, nzm, o.skip, st);
  else
    return launch_ystd_pt<T, TS, BC, FWD, PTM>(data, nx, ny, nplanes, tab, lines, nzm, o, st);
}

template <typename T, typename TS, int BC, bool FWD>
static hipError_t launch_y_bc(TS* data, int nx, int ny, int nplanes, const T* tab, int pt,
                              const PassOpts& o, hipStream_t st) {
  return pt == 8 ? launch_y_pt<T, TS, BC, FWD, 8>(data, nx, ny, nplanes, tab, o, st)
                 : launch_y_pt<T, TS, BC, FWD, 16>(data, nx, ny, nplanes, tab, o, st);
}

#if VP_IN_PART(1)
hipError_t launch_y_f64(double* data, int nx, int ny, int nplanes, int bc, bool fwd,
                        const double* tab, int pt, int lines, hipStream_t st) {
  PassOpts o{};
  o.lines = lines;
  return with_bc(bc, [&](auto B) {
    constexpr int BC = decltype(B)::value;
    return fwd ? launch_y_bc<double, double, BC, true>(data, nx, ny, nplanes, tab, pt, o, st)
               : launch_y_bc<double, double, BC, false>(data, nx, ny, nplanes, tab, pt, o, st);
  });
}
#endif

#if VP_IN_PART(2)
hipError_t launch_y_f32(float* data, int nx, int ny, int nplanes, int bc, bool fwd,
                        const double* tab, int pt, const PassOpts& o, hipStream_t st) {
  return with_bc(bc, [&](auto B) {
    constexpr int BC = decltype(B)::value;
    return fwd ? launch_y_bc<double, float, BC, true>(data, nx, ny, nplanes, tab, pt, o, st)
               : launch_y_bc<double, float, BC, false>(data, nx, ny, nplanes, tab, pt, o, st);
  });
}
#endif

}  // namespace vp
