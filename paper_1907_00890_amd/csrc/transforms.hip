// x and y passes of the spectral Poisson solve: real-to-real transforms of
// every x-line (contiguous rows) and every y-line (columns of a z-plane).
//
// x pass: a block owns RPB = 4096/N consecutive rows (one contiguous chunk
// of 4096 values), pairs them as (re, im) lines and transforms 2 real rows
// with one complex FFT.  y pass: a block owns a tile of C consecutive columns
// of one z-plane, pairs neighbouring columns the same way; each row of the
// tile is one C-wide contiguous chunk in memory.  Both passes stage the
// block's data in LDS, so global loads and stores stay coalesced.
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"
#include "kernels.hpp"

namespace vp {

// ---------------------------------------------------------------------------
// x pass
// ---------------------------------------------------------------------------
template <typename TI, typename T, typename TO, int N, int BC, bool FWD, bool ACCUM>
__global__ __launch_bounds__(256) void k_xpass(const TI* __restrict__ in, TO* __restrict__ out,
                                                long nrows, const T* __restrict__ tab,
                                                const double* __restrict__ sub) {
  constexpr int TPL = N / 8;
  constexpr int LPB = 256 / TPL;  // complex lines per block
  constexpr int RPB = 2 * LPB;    // real rows per block
  constexpr int LD = N + 1;       // padded LDS row stride
  __shared__ T lds[RPB * LD];
  const int tid = threadIdx.x;
  const long row0 = (long)blockIdx.x * RPB;
  const long nval = (nrows - row0 < RPB ? nrows - row0 : RPB) * (long)N;
  const long g0 = row0 * N;

#pragma unroll 4
  for (int e = tid; e < RPB * N; e += 256) {
    const int r = e / N, c = e % N;
    lds[r * LD + c] = e < nval ? T(in[g0 + e]) : T(0);
  }
  __syncthreads();

  const int q = tid / TPL, t = tid % TPL;
  T* a = lds + (2 * q) * LD;
  T* b = lds + (2 * q + 1) * LD;
  const T* twc = tab;
  const T* tws = tab + N;
  const T* pc = tab + 2 * N;
  const T* ps = tab + 2 * N + (N / 2 + 1);
  if constexpr (FWD)
    real_pair_forward<T, N, BC, TPL>(a, b, 1, t, twc, tws, pc, ps);
  else
    real_pair_inverse<T, N, BC, TPL>(a, b, 1, t, twc, tws, pc, ps);

  TO shift = TO(0);
  if constexpr (ACCUM) {
    if (sub) shift = TO(sub[0]);
  }
#pragma unroll 4
  for (int e = tid; e < RPB * N; e += 256) {
    if (e < nval) {
      const int r = e / N, c = e % N;
      if constexpr (ACCUM)
        out[g0 + e] += TO(lds[r * LD + c]) - shift;
      else
        out[g0 + e] = TO(lds[r * LD + c]);
    }
  }
}

// ---------------------------------------------------------------------------
// y pass: block (tile, plane); tile = C columns x N rows, threads = (C/2)*(N/8)
// ---------------------------------------------------------------------------
template <typename T, int N, int BC, bool FWD>
__global__ __launch_bounds__(1024) void k_ypass(T* __restrict__ data, int nx, long plane, int C,
                                                 const T* __restrict__ tab) {
  constexpr int TPL = N / 8;
  extern __shared__ unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);
  const int CS = C + 1;  // padded tile row stride
  const int nthr = (C / 2) * TPL;
  const int tid = threadIdx.x;
  const long base = (long)blockIdx.y * plane + (long)blockIdx.x * C;

  for (int e = tid; e < N * C; e += nthr) {
    const int j = e / C, c = e % C;
    tile[j * CS + c] = data[base + (long)j * nx + c];
  }
  __syncthreads();

  const int p = tid % (C / 2), t = tid / (C / 2);
  T* a = tile + 2 * p;
  T* b = tile + 2 * p + 1;
  const T* twc = tab;
  const T* tws = tab + N;
  const T* pc = tab + 2 * N;
  const T* ps = tab + 2 * N + (N / 2 + 1);
  if constexpr (FWD)
    real_pair_forward<T, N, BC, TPL>(a, b, CS, t, twc, tws, pc, ps);
  else
    real_pair_inverse<T, N, BC, TPL>(a, b, CS, t, twc, tws, pc, ps);

  for (int e = tid; e < N * C; e += nthr) {
    const int j = e / C, c = e % C;
    data[base + (long)j * nx + c] = tile[j * CS + c];
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <typename TI, typename T, typename TO, int BC, bool FWD, bool ACCUM>
static hipError_t launch_x_bc(const void* in, void* out, int n, long nrows, const void* tab,
                              const double* sub, hipStream_t st) {
  const long rpb = 2 * (256 / (n / 8));
  const dim3 grid((unsigned)((nrows + rpb - 1) / rpb));
  const TI* i = static_cast<const TI*>(in);
  TO* o = static_cast<TO*>(out);
  const T* tb = static_cast<const T*>(tab);
#define VP_XCASE(NN)                                                                     \
  case NN:                                                                               \
    hipLaunchKernelGGL((k_xpass<TI, T, TO, NN, BC, FWD, ACCUM>), grid, dim3(256), 0, st, \
                       i, o, nrows, tb, sub);                                            \
    break;
  switch (n) {
    VP_XCASE(8) VP_XCASE(16) VP_XCASE(32) VP_XCASE(64) VP_XCASE(128) VP_XCASE(256)
    VP_XCASE(512) VP_XCASE(1024)
    default: return hipErrorInvalidValue;
  }
#undef VP_XCASE
  return hipGetLastError();
}

template <typename TI, typename T, typename TO, bool FWD, bool ACCUM>
static hipError_t launch_x(const void* in, void* out, int n, int bc, long nrows, const void* tab,
                           hipStream_t st, const double* sub = nullptr) {
  return bc == BC_P ? launch_x_bc<TI, T, TO, BC_P, FWD, ACCUM>(in, out, n, nrows, tab, sub, st)
                    : launch_x_bc<TI, T, TO, BC_N, FWD, ACCUM>(in, out, n, nrows, tab, sub, st);
}

int ypass_tile_cols(int nx, int ny) {
  int c = 4096 / ny;
  if (c < 16) c = 16;
  if (c > nx) c = nx;
  return c;
}

template <typename T, int BC, bool FWD>
static hipError_t launch_y_bc(void* data, int nx, int ny, int nz, const void* tab, hipStream_t st) {
  const int C = ypass_tile_cols(nx, ny);
  const int nthr = (C / 2) * (ny / 8);
  const size_t shm = sizeof(T) * (size_t)ny * (C + 1);
  const dim3 grid((unsigned)(nx / C), (unsigned)nz);
  T* d = static_cast<T*>(data);
  const T* tb = static_cast<const T*>(tab);
  const long plane = (long)nx * ny;
#define VP_YCASE(NN)                                                                        \
  case NN:                                                                                  \
    if (shm > 65536) {                                                                      \
      const hipError_t e = allow_large_lds(&k_ypass<T, NN, BC, FWD>);                       \
      if (e != hipSuccess) return e;                                                        \
    }                                                                                       \
    hipLaunchKernelGGL((k_ypass<T, NN, BC, FWD>), grid, dim3(nthr), shm, st, d, nx, plane, C, \
                       tb);                                                                 \
    break;
  switch (ny) {
    VP_YCASE(8) VP_YCASE(16) VP_YCASE(32) VP_YCASE(64) VP_YCASE(128) VP_YCASE(256)
    VP_YCASE(512) VP_YCASE(1024)
    default: return hipErrorInvalidValue;
  }
#undef VP_YCASE
  return hipGetLastError();
}

hipError_t launch_xfwd_f64(const double* in, double* out, int nx, int bc, long nrows,
                           const double* tab, hipStream_t st) {
  return launch_x<double, double, double, true, false>(in, out, nx, bc, nrows, tab, st);
}
hipError_t launch_xinv_f64(const double* in, double* out, int nx, int bc, long nrows,
                           const double* tab, hipStream_t st) {
  return launch_x<double, double, double, false, false>(in, out, nx, bc, nrows, tab, st);
}
hipError_t launch_xfwd_f32(const double* in, float* out, int nx, int bc, long nrows,
                           const float* tab, hipStream_t st) {
  return launch_x<double, float, float, true, false>(in, out, nx, bc, nrows, tab, st);
}
hipError_t launch_xinv_f32(const float* in, double* out, int nx, int bc, long nrows, bool accum,
                           const double* sub, const float* tab, hipStream_t st) {
  return accum ? launch_x<float, float, double, false, true>(in, out, nx, bc, nrows, tab, st, sub)
               : launch_x<float, float, double, false, false>(in, out, nx, bc, nrows, tab, st);
}
hipError_t launch_y_f64(double* data, int nx, int ny, int nz, int bc, bool fwd, const double* tab,
                        hipStream_t st) {
  if (bc == BC_P)
    return fwd ? launch_y_bc<double, BC_P, true>(data, nx, ny, nz, tab, st)
               : launch_y_bc<double, BC_P, false>(data, nx, ny, nz, tab, st);
  return fwd ? launch_y_bc<double, BC_N, true>(data, nx, ny, nz, tab, st)
             : launch_y_bc<double, BC_N, false>(data, nx, ny, nz, tab, st);
}
hipError_t launch_y_f32(float* data, int nx, int ny, int nz, int bc, bool fwd, const float* tab,
                        hipStream_t st) {
  if (bc == BC_P)
    return fwd ? launch_y_bc<float, BC_P, true>(data, nx, ny, nz, tab, st)
               : launch_y_bc<float, BC_P, false>(data, nx, ny, nz, tab, st);
  return fwd ? launch_y_bc<float, BC_N, true>(data, nx, ny, nz, tab, st)
             : launch_y_bc<float, BC_N, false>(data, nx, ny, nz, tab, st);
}

}  // namespace vp
