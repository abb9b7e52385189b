// Spectral z pass of a uniform z grid: forward transform along z, division
// by the three-dimensional eigenvalue, inverse transform, in one LDS pass.
#include "transform_passes.hpp"

namespace vp {

// ---------------------------------------------------------------------------
// spectral z pass (uniform z): block (tile, member); tile = 2*lines
// consecutive (kx, ky) positions of the plane, each a z-line of N values
// `plane` apart.  Per packed z coefficient c of line (kx, ky):
//   x <- x * scale / (lamx[kx] + lamy[ky] + lamz[c]),  0 where that is 0
// (only the constant mode), which is the pseudo-inverse; the removed
// constant (the coefficient times scale: the mean) goes to mean_out[member].
// T: arithmetic and LDS type; TS: type of the data in HBM.
// ---------------------------------------------------------------------------
template <typename T, typename TS, int N, int BC, int PTM>
__global__ __launch_bounds__(PTM == 8 ? 512 : 256) void k_zspec(
    TS* __restrict__ data, int nx, long plane, int llines, const T* __restrict__ tab,
    const double* __restrict__ lamx, const double* __restrict__ lamy,
    const double* __restrict__ lamz, double scale, long batch_stride,
    double* __restrict__ mean_out, const int* __restrict__ skip) {
  using T2 = typename Vec2<T>::type;
  using S2 = typename Vec2<TS>::type;
  extern __shared__ unsigned char smem_raw[];
  if (skip && skip[blockIdx.y]) return;  // member already converged (whole block)
  const int lines = 1 << llines;
  const int q = threadIdx.x & (lines - 1), t = threadIdx.x >> llines;
  const long pos = (long)xcd_tile(blockIdx.x, gridDim.x) * 2 * lines + 2 * q;  // line a; b: pos + 1
  S2* col = reinterpret_cast<S2*>(data + blockIdx.y * batch_stride + pos);
  const long pstride = plane >> 1;  // z stride in S2 units
  const double la = lamx[pos % nx] + lamy[pos / nx];
  const double lb = lamx[(pos + 1) % nx] + lamy[(pos + 1) / nx];
  YLds<T, N> lds(reinterpret_cast<T2*>(smem_raw), q, lines);
  spectral_body<T, N, BC, PTM>(
      lds, t, tab,
      [&](int e, T& r, T& i) {
        const S2 v = col[(long)e * pstride];
        r = T(v.x);
        i = T(v.y);
      },
      [&](int c, T& a, T& b) {
        const double lz = lamz[c];
        const double da = la + lz, db = lb + lz;
        if (da == 0.0) {
          if (mean_out && c == 0) mean_out[blockIdx.y] = double(a) * scale;
          a = T(0);
        } else {
          a = T(double(a) * (scale / da));
        }
        b = T(double(b) * (scale / db));
      },
      [&](int e, T r, T i) {
        S2 v;
        v.x = TS(r);
        v.y = TS(i);
        col[(long)e * pstride] = v;
      });
}

template <typename T, typename TS, int BC, int PTM>
static hipError_t launch_zspec_pt(TS* data, const ZSpecArgs& a, const T* tab, int nb,
                                  const int* skip, hipStream_t st) {
  using T2 = typename Vec2<T>::type;
  const long plane = (long)a.nx * a.ny;
  // tile width: as for the y pass of a line of the same length, or a.lines
  int lines = pass_threads(a.nz) / fft_tpl(a.nz);
  if (a.lines > 0 && a.lines < lines) lines = a.lines;
  if (lines > pow2_part(plane) / 2) lines = (int)(pow2_part(plane) / 2);  // tiles divide the plane
  int ll = 0;
  while ((1 << ll) < lines) ++ll;
  if (nb < 1 || nb > kMaxBatch) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(plane / (2 * lines)), (unsigned)nb);
#define VP_ZS(NN)                                                                          \
  case NN: {                                                                               \
    const int nthr = lines * FftShape<NN, PTM>::TPL;                                       \
    const size_t shm = sizeof(T2) * (size_t)lds_len<NN>() * (lines + 1);                   \
    auto kern = &k_zspec<T, TS, NN, BC, canon_ptm<NN, PTM>()>;                                 \
    if (shm > 65536) {                                                                     \
      const hipError_t e = allow_large_lds(kern);                                          \
      if (e != hipSuccess) return e;                                                       \
    }                                                                                      \
    hipLaunchKernelGGL(kern, grid, dim3(nthr), shm, st, data, a.nx, plane, ll, tab,        \
                       a.lamx, a.lamy, a.lamz, a.scale, a.batch_stride, a.mean_out, skip); \
    break;                                                                                 \
  }
  switch (a.nz) {
    VP_SIZES(VP_ZS)
    default: return hipErrorInvalidValue;
  }
#undef VP_ZS
  return hipGetLastError();
}

template <typename T, typename TS>
static hipError_t launch_zspec_t(TS* data, const ZSpecArgs& a, const T* tab, int pt, int nb,
                                 const int* skip, hipStream_t st) {
  return with_bc(a.bcz, [&](auto B) -> hipError_t {
    constexpr int BC = decltype(B)::value;
    if constexpr (BC == BC_ND || BC == BC_DN)
      return hipErrorInvalidValue;  // the tridiagonal pass takes these
    else
      return pt == 8 ? launch_zspec_pt<T, TS, BC, 8>(data, a, tab, nb, skip, st)
                     : launch_zspec_pt<T, TS, BC, 16>(data, a, tab, nb, skip, st);
  });
}

#if VP_IN_PART(1)
hipError_t launch_zspec_f64(double* data, const ZSpecArgs& a, const double* tab, int pt, int nb,
                            hipStream_t st) {
  return launch_zspec_t<double, double>(data, a, tab, pt, nb, nullptr, st);
}
#endif

#if VP_IN_PART(2)
hipError_t launch_zspec_f32(float* data, const ZSpecArgs& a, const double* tab, int pt, int nb,
                            const int* skip, hipStream_t st) {
  return launch_zspec_t<double, float>(data, a, tab, pt, nb, skip, st);
}
#endif

}  // namespace vp
