// x and y passes of the spectral Poisson solve: real-to-real transforms of
// every x-line (contiguous rows) and every y-line (columns of a z-plane), two
// real lines per complex FFT (see fft_lds.hpp for the packed spectra).
//
// Data path of a forward pass: the first Stockham pass loads straight from
// HBM into registers (a line's N/16 threads read consecutive addresses), the
// intermediate passes exchange through LDS, and the real-pair step reads the
// last pass from LDS and writes the packed spectrum straight to HBM.  The
// inverse mirrors it: the real-pair step loads from HBM into LDS and the last
// Stockham pass stores to HBM.  One block owns 2*LPB whole rows (x) or a
// tile of 2*LINES columns of one z-plane (y), so every HBM access is a
// contiguous chunk.  LDS rows are padded by one slot every 16 values, which
// spreads the strided writes of the first pass over the banks.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_lds.hpp"
#include "kernels.hpp"

namespace vp {

__device__ __forceinline__ int lds_pos(int e) { return e + (e >> 4); }
template <int N>
constexpr int lds_len() {
  return N + N / 16 + 1;
}

// ---------------------------------------------------------------------------
// LDS access policies: x lines as separate re/im rows, y lines interleaved
// ---------------------------------------------------------------------------
template <typename T, int N>
struct XLds {
  T* re;
  T* im;
  __device__ XLds(T* base, int q, int lpb) {
    re = base + q * lds_len<N>();
    im = base + (lpb + q) * lds_len<N>();
  }
  __device__ void put(int e, T r, T i) {
    re[lds_pos(e)] = r;
    im[lds_pos(e)] = i;
  }
  __device__ void get(int e, T& r, T& i) const {
    r = re[lds_pos(e)];
    i = im[lds_pos(e)];
  }
};

template <typename T, int N>
struct YLds {
  using T2 = typename Vec2<T>::type;
  T2* base;
  int lp;
  __device__ YLds(T2* b, int q, int lines) : base(b + q), lp(lines + 1) {}
  __device__ void put(int e, T r, T i) {
    T2 v;
    v.x = r;
    v.y = i;
    base[lds_pos(e) * lp] = v;
  }
  __device__ void get(int e, T& r, T& i) const {
    const T2 v = base[lds_pos(e) * lp];
    r = v.x;
    i = v.y;
  }
};

// Stockham passes after the first one, through LDS (in place).  With
// LAST_IN_REGS the last pass stays in registers (the caller stores it);
// otherwise it is written back to LDS.  Twiddle loads are issued before the
// barrier they wait on.
template <typename T, int N, int NS, int SIGN, bool LAST_IN_REGS, int PTM, typename L>
__device__ __forceinline__ void later_passes(L& lds, int t, const T* __restrict__ tab, T* vr,
                                             T* vi) {
  if constexpr (NS < N) {
    constexpr int R = PassRadix<N, NS, PTM>::R;
    constexpr int B = FftShape<N, PTM>::PT / R;
    constexpr bool LAST = (NS * R == N);
    T wr[FftShape<N, PTM>::PT], wi[FftShape<N, PTM>::PT];
    if constexpr (NS > 1) load_twiddles<T, N, NS, SIGN, PTM>(tab, t, wr, wi);
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) lds.get(pass_in<N, NS, PTM>(t, b, r), vr[b * R + r], vi[b * R + r]);
    __syncthreads();
    pass_compute<T, N, NS, SIGN, PTM>(vr, vi, wr, wi);
    if constexpr (!(LAST && LAST_IN_REGS)) {
#pragma unroll
      for (int b = 0; b < B; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) lds.put(pass_out<N, NS, PTM>(t, b, r), vr[b * R + r], vi[b * R + r]);
    }
    later_passes<T, N, NS * R, SIGN, LAST_IN_REGS, PTM>(lds, t, tab, vr, vi);
  }
}

// Outflow at both ends (BC_D): the sine transform (DST-II) of a line is the
// cosine transform (DCT-II) of the line with every odd element negated, read
// in reverse order: DST_k(x) = DCT_{N-1-k}((-1)^i x_i).  The forward pass
// negates odd elements on load and the inverse negates them on store; the
// packed coefficient c then belongs to sine mode N-1-c (the eigenvalue
// tables are indexed by c accordingly).
template <typename T>
__device__ __forceinline__ void flip_odd(int e, T& re, T& im) {
  if (e & 1) {
    re = -re;
    im = -im;
  }
}

// stride NS of the last pass of the plan for length N
template <int N, int PTM, int NS = 1>
constexpr int last_ns() {
  if constexpr (NS * PassRadix<N, NS, PTM>::R == N) return NS;
  else return last_ns<N, PTM, NS * PassRadix<N, NS, PTM>::R>();
}

// ---------------------------------------------------------------------------
// forward pass body shared by x and y: `load(e, re, im)` gives element e of
// lines a and b; `store(c0, a0, b0, c1, a1, b1)` writes packed coefficients
// c0 and c1 of both lines
// ---------------------------------------------------------------------------
template <typename T, int N, int BC, int PTM, typename L, typename Load, typename Store>
__device__ __forceinline__ void forward_body(L& lds, int t, const T* __restrict__ tab, Load load,
                                             Store store) {
  using S = FftShape<N, PTM>;
  constexpr int PT = S::PT, TPL = S::TPL;
  constexpr int R1 = PassRadix<N, 1, PTM>::R;
  T vr[PT], vi[PT];
#pragma unroll
  for (int r = 0; r < PT; ++r) {
    // inputs of the first pass's butterflies (t + r TPL when a thread holds one)
    int e = pass_in<N, 1, PTM>(t, r / R1, r % R1);
    if constexpr (BC != BC_P) e = dct_perm<N>(e);
    load(e, vr[r], vi[r]);
    if constexpr (BC == BC_D) flip_odd(e, vr[r], vi[r]);
  }
  {
    T wr[PT], wi[PT];
    pass_compute<T, N, 1, -1, PTM>(vr, vi, wr, wi);
  }
#pragma unroll
  for (int b = 0; b < PT / R1; ++b)
#pragma unroll
    for (int r = 0; r < R1; ++r)
      lds.put(pass_out<N, 1, PTM>(t, b, r), vr[b * R1 + r], vi[b * R1 + r]);
  later_passes<T, N, R1, -1, false, PTM>(lds, t, tab, vr, vi);
  __syncthreads();
  // (cos, sin)(pi m/(2N)) pairs of the DCT rotation
  const typename Vec2<T>::type* rot = reinterpret_cast<const typename Vec2<T>::type*>(tab) + N;
#pragma unroll
  for (int u = 0; u < PT / 2; ++u) {
    const int m = t + TPL * u;
    T zr, zi;
    lds.get(m, zr, zi);
    if (m == 0) {
      T hr, hi;
      lds.get(N / 2, hr, hi);
      if constexpr (BC == BC_P) {
        store(0, zr, zi, 1, hr, hi);
      } else {
        const T h = T(0.70710678118654752440084436210485);
        store(0, zr, zi, N / 2, h * hr, h * hi);
      }
    } else {
      T wr, wi;
      lds.get(N - m, wr, wi);
      T oa[2], ob[2];
      RealPair<T, N, BC>::post(zr, zi, wr, wi, rot[m].x, rot[m].y, oa, ob);
      if constexpr (BC == BC_P)
        store(2 * m, oa[0], ob[0], 2 * m + 1, oa[1], ob[1]);
      else
        store(m, oa[0], ob[0], N - m, oa[1], ob[1]);
    }
  }
}

// inverse body: `load2(c0, c1, a0, b0, a1, b1)` reads packed coefficients c0
// and c1 of both lines; `store(e, re, im)` writes element e of lines a and b
template <typename T, int N, int BC, int PTM, typename L, typename Load2, typename Store>
__device__ __forceinline__ void inverse_body(L& lds, int t, const T* __restrict__ tab, Load2 load2,
                                             Store store) {
  using S = FftShape<N, PTM>;
  constexpr int PT = S::PT, TPL = S::TPL;
  // (cos, sin)(pi m/(2N)) pairs of the DCT rotation
  const typename Vec2<T>::type* rot = reinterpret_cast<const typename Vec2<T>::type*>(tab) + N;
#pragma unroll
  for (int u = 0; u < PT / 2; ++u) {
    const int m = t + TPL * u;
    if (m == 0) {
      T a0, b0, a1, b1;
      if constexpr (BC == BC_P) {
        load2(0, 1, a0, b0, a1, b1);
      } else {
        load2(0, N / 2, a0, b0, a1, b1);
        const T r2 = T(1.4142135623730950488016887242097);
        a1 *= r2;
        b1 *= r2;
      }
      lds.put(0, a0, b0);
      lds.put(N / 2, a1, b1);
    } else {
      T ia[2], ib[2];
      if constexpr (BC == BC_P)
        load2(2 * m, 2 * m + 1, ia[0], ib[0], ia[1], ib[1]);
      else
        load2(m, N - m, ia[0], ib[0], ia[1], ib[1]);
      T z0r, z0i, z1r, z1i;
      RealPair<T, N, BC>::pre(ia, ib, rot[m].x, rot[m].y, z0r, z0i, z1r, z1i);
      lds.put(m, z0r, z0i);
      lds.put(N - m, z1r, z1i);
    }
  }
  T vr[PT], vi[PT];
  later_passes<T, N, 1, +1, true, PTM>(lds, t, tab, vr, vi);
  // the last pass is in registers: store to HBM
  constexpr int NSL = last_ns<N, PTM>();
  constexpr int RL = PassRadix<N, NSL, PTM>::R;
#pragma unroll
  for (int b = 0; b < PT / RL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int e = pass_out<N, NSL, PTM>(t, b, r);
      if constexpr (BC != BC_P) e = dct_perm<N>(e);
      if constexpr (BC == BC_D) flip_odd(e, vr[b * RL + r], vi[b * RL + r]);
      store(e, vr[b * RL + r], vi[b * RL + r]);
    }
}

// ---------------------------------------------------------------------------
// forward transform, per-coefficient scaling, inverse transform of two real
// lines held in LDS, in one pass: `load(e, re, im)` gives element e of lines
// a and b; `scale(c, a, b)` rescales the packed coefficient c of both lines
// in place; `store(e, re, im)` writes element e.  Between the two transforms
// a thread reads and writes only the LDS positions of its own modes m and
// N - m (and N/2 for m = 0), so no barrier is needed there.
// ---------------------------------------------------------------------------
template <typename T, int N, int BC, int PTM, typename L, typename Load, typename Scale,
          typename Store>
__device__ __forceinline__ void spectral_body(L& lds, int t, const T* __restrict__ tab, Load load,
                                              Scale scale, Store store) {
  using S = FftShape<N, PTM>;
  constexpr int PT = S::PT, TPL = S::TPL;
  constexpr int R1 = PassRadix<N, 1, PTM>::R;
  T vr[PT], vi[PT];
#pragma unroll
  for (int r = 0; r < PT; ++r) {
    // inputs of the first pass's butterflies (t + r TPL when a thread holds one)
    int e = pass_in<N, 1, PTM>(t, r / R1, r % R1);
    if constexpr (BC != BC_P) e = dct_perm<N>(e);
    load(e, vr[r], vi[r]);
    if constexpr (BC == BC_D) flip_odd(e, vr[r], vi[r]);
  }
  {
    T wr[PT], wi[PT];
    pass_compute<T, N, 1, -1, PTM>(vr, vi, wr, wi);
  }
#pragma unroll
  for (int b = 0; b < PT / R1; ++b)
#pragma unroll
    for (int r = 0; r < R1; ++r)
      lds.put(pass_out<N, 1, PTM>(t, b, r), vr[b * R1 + r], vi[b * R1 + r]);
  later_passes<T, N, R1, -1, false, PTM>(lds, t, tab, vr, vi);
  __syncthreads();
  // (cos, sin)(pi m/(2N)) pairs of the DCT rotation
  const typename Vec2<T>::type* rot = reinterpret_cast<const typename Vec2<T>::type*>(tab) + N;
#pragma unroll
  for (int u = 0; u < PT / 2; ++u) {
    const int m = t + TPL * u;
    T zr, zi;
    lds.get(m, zr, zi);
    if (m == 0) {
      T hr, hi;
      lds.get(N / 2, hr, hi);
      // packed coefficients 0 and 1 (periodic) or 0 and N/2 (walls, outflow)
      T a0 = zr, b0 = zi, a1 = hr, b1 = hi;
      int c1 = 1;
      if constexpr (BC != BC_P) {
        const T h = T(0.70710678118654752440084436210485);
        a1 *= h;
        b1 *= h;
        c1 = N / 2;
      }
      scale(0, a0, b0);
      scale(c1, a1, b1);
      if constexpr (BC != BC_P) {
        const T r2 = T(1.4142135623730950488016887242097);
        a1 *= r2;
        b1 *= r2;
      }
      lds.put(0, a0, b0);
      lds.put(N / 2, a1, b1);
    } else {
      T wr, wi;
      lds.get(N - m, wr, wi);
      T oa[2], ob[2];
      RealPair<T, N, BC>::post(zr, zi, wr, wi, rot[m].x, rot[m].y, oa, ob);
      const int c0 = BC == BC_P ? 2 * m : m, c1 = BC == BC_P ? 2 * m + 1 : N - m;
      scale(c0, oa[0], ob[0]);
      scale(c1, oa[1], ob[1]);
      T z0r, z0i, z1r, z1i;
      RealPair<T, N, BC>::pre(oa, ob, rot[m].x, rot[m].y, z0r, z0i, z1r, z1i);
      lds.put(m, z0r, z0i);
      lds.put(N - m, z1r, z1i);
    }
  }
  later_passes<T, N, 1, +1, true, PTM>(lds, t, tab, vr, vi);
  constexpr int NSL = last_ns<N, PTM>();
  constexpr int RL = PassRadix<N, NSL, PTM>::R;
#pragma unroll
  for (int b = 0; b < PT / RL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      int e = pass_out<N, NSL, PTM>(t, b, r);
      if constexpr (BC != BC_P) e = dct_perm<N>(e);
      if constexpr (BC == BC_D) flip_odd(e, vr[b * RL + r], vi[b * RL + r]);
      store(e, vr[b * RL + r], vi[b * RL + r]);
    }
}

// ---------------------------------------------------------------------------
// A wall at one end and an outflow at the other (BC_ND: wall at the lower
// end, BC_DN: at the upper): the eigenvectors of the second difference are
// the quarter-wave cosines cos(pi (2k+1)(2i+1)/(4N)), i.e. the DCT-IV (for
// BC_DN the same on the reversed line).  A DCT-IV of one real line of
// length N is one complex FFT of length H = N/2:
//   v_e = (x_{2e} + i x_{N-1-2e}) e^{-i pi (4e+1)/(4N)},  V = FFT_H(v),
//   W_k = V_k e^{-i pi k/N},  X_{2k} = Re W_k,  X_{N-1-2k} = -Im W_k,
// and the DCT-IV is its own inverse up to the factor N/2.  `load(e, v)`
// gives element e of the line, `store(c, v)` writes element c of the
// result.  tab: (cos, sin) pairs of 2 pi j/H for j < H, then of
// pi (4e+1)/(4N) for e < H, then of pi k/N for k < H.
// ---------------------------------------------------------------------------
template <typename T, int N, int PTM, typename L, typename Load, typename Store>
__device__ __forceinline__ void quarter_body(L& lds, int t, const T* __restrict__ tab, Load load,
                                             Store store) {
  constexpr int H = N / 2;
  using S = FftShape<H, PTM>;
  constexpr int PT = S::PT, TPL = S::TPL;
  constexpr int R1 = PassRadix<H, 1, PTM>::R;
  using T2 = typename Vec2<T>::type;
  const T2* pre = reinterpret_cast<const T2*>(tab) + H;
  const T2* post = pre + H;
  T vr[PT], vi[PT];
#pragma unroll
  for (int r = 0; r < PT; ++r) {
    const int e = pass_in<H, 1, PTM>(t, r / R1, r % R1);  // first-pass butterfly inputs
    T a, b;
    load(2 * e, a);
    load(N - 1 - 2 * e, b);
    const T2 w = pre[e];
    vr[r] = a * w.x + b * w.y;  // (a + i b)(cos - i sin)
    vi[r] = b * w.x - a * w.y;
  }
  {
    T wr[PT], wi[PT];
    pass_compute<T, H, 1, -1, PTM>(vr, vi, wr, wi);
  }
  if constexpr (R1 < H) {
#pragma unroll
    for (int b = 0; b < PT / R1; ++b)
#pragma unroll
      for (int r = 0; r < R1; ++r)
        lds.put(pass_out<H, 1, PTM>(t, b, r), vr[b * R1 + r], vi[b * R1 + r]);
    later_passes<T, H, R1, -1, true, PTM>(lds, t, tab, vr, vi);
  }
  constexpr int NSL = last_ns<H, PTM>();
  constexpr int RL = PassRadix<H, NSL, PTM>::R;
#pragma unroll
  for (int b = 0; b < PT / RL; ++b)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int k = pass_out<H, NSL, PTM>(t, b, r);
      const T2 w = post[k];
      const T xr = vr[b * RL + r], xi = vi[b * RL + r];
      store(2 * k, xr * w.x + xi * w.y);
      store(N - 1 - 2 * k, -(xi * w.x - xr * w.y));
    }
}

// physical position of element e of a line for the quarter-wave transform
template <int N, int BC>
__device__ __forceinline__ int qpos(int e) {
  return BC == BC_DN ? N - 1 - e : e;
}

// ---------------------------------------------------------------------------
// x kernels: a block owns 2*LPB consecutive rows (nrows is even)
// ---------------------------------------------------------------------------
// SUB: member b's input is read as in[b] - sub[b] (FP64, before any
// conversion to T); without it the kernel reads its input unchanged.
template <typename TI, typename T, int N, int BC, bool SUB, int PTM>
__global__ __launch_bounds__(256) void k_xfwd(const Batch<const TI> in, T* __restrict__ out,
                                               long ostride, long nrows,
                                               const T* __restrict__ tab,
                                               const double* __restrict__ sub,
                                               const int* __restrict__ skip) {
  constexpr int TPL = FftShape<N, PTM>::TPL, LPB = 256 / TPL;
  __shared__ T lds_mem[2 * LPB * lds_len<N>()];
  if (skip && skip[blockIdx.y]) return;  // member already converged (whole block)
  const int q = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long ra = (long)blockIdx.x * 2 * LPB + 2 * q;
  const bool ok = ra < nrows;
  const TI* ga = in.p[blockIdx.y] + ra * N;
  const TI* gb = ga + N;
  T* oa = out + blockIdx.y * ostride + ra * N;
  T* ob = oa + N;
  TI shift = TI(0);
  if constexpr (SUB) shift = TI(sub[blockIdx.y]);
  XLds<T, N> lds(lds_mem, q, LPB);
  forward_body<T, N, BC, PTM>(
      lds, t, tab,
      [&](int e, T& r, T& i) {
        if constexpr (SUB) {
          r = ok ? T(ga[e] - shift) : T(0);
          i = ok ? T(gb[e] - shift) : T(0);
        } else {
          r = ok ? T(ga[e]) : T(0);
          i = ok ? T(gb[e]) : T(0);
        }
      },
      [&](int c0, T a0, T b0, int c1, T a1, T b1) {
        if (!ok) return;
        oa[c0] = a0;
        ob[c0] = b0;
        oa[c1] = a1;
        ob[c1] = b1;
      });
}

// With FP32 input (the mixed chain) and `norms` set, each block also writes
// the sums of e^2 and p^2 over its rows to norms[2 * (member * gridDim.x +
// block) + {0, 1}], where e is the value added (or stored) and p the result.
template <typename T, typename TO, int N, int BC, bool ACCUM, int PTM>
__global__ __launch_bounds__(256) void k_xinv(const T* __restrict__ in, long istride,
                                               const Batch<TO> out, long nrows,
                                               const T* __restrict__ tab,
                                               const double* __restrict__ sub,
                                               const int* __restrict__ skip,
                                               double* __restrict__ norms) {
  constexpr int TPL = FftShape<N, PTM>::TPL, LPB = 256 / TPL;
  constexpr bool NORMS = !std::is_same<T, TO>::value;
  __shared__ T lds_mem[2 * LPB * lds_len<N>()];
  if (skip && skip[blockIdx.y]) return;  // member already converged (whole block)
  double ee = 0.0, pp = 0.0;
  const int q = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long ra = (long)blockIdx.x * 2 * LPB + 2 * q;
  const bool ok = ra < nrows;
  const T* ia = in + blockIdx.y * istride + ra * N;
  const T* ib = ia + N;
  TO* oa = out.p[blockIdx.y] + ra * N;
  TO* ob = oa + N;
  TO shift = TO(0);
  if constexpr (ACCUM) {
    if (sub) shift = TO(sub[blockIdx.y]);
  }
  XLds<T, N> lds(lds_mem, q, LPB);
  inverse_body<T, N, BC, PTM>(
      lds, t, tab,
      [&](int c0, int c1, T& a0, T& b0, T& a1, T& b1) {
        a0 = ok ? ia[c0] : T(0);
        b0 = ok ? ib[c0] : T(0);
        a1 = ok ? ia[c1] : T(0);
        b1 = ok ? ib[c1] : T(0);
      },
      [&](int e, T r, T i) {
        if (!ok) return;
        const TO da = TO(r) - shift, db = TO(i) - shift;
        TO pa = da, pb = db;
        if constexpr (ACCUM) {
          pa = oa[e] + da;
          pb = ob[e] + db;
        }
        oa[e] = pa;
        ob[e] = pb;
        if constexpr (NORMS) {
          ee += double(da) * double(da) + double(db) * double(db);
          pp += double(pa) * double(pa) + double(pb) * double(pb);
        }
      });
  if constexpr (NORMS) {
    if (norms) {
      // fixed-order block reduction through the (now free) LDS of the transform
      double* red = reinterpret_cast<double*>(lds_mem);
      __syncthreads();
      red[threadIdx.x] = ee;
      red[256 + threadIdx.x] = pp;
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
          red[threadIdx.x] += red[threadIdx.x + w];
          red[256 + threadIdx.x] += red[256 + threadIdx.x + w];
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        const long o = 2 * ((long)blockIdx.y * gridDim.x + blockIdx.x);
        norms[o] = red[0];
        norms[o + 1] = red[256];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// y kernels: block (tile, plane); tile = 2*lines columns x N rows; thread
// (q, t) with q fastest, so a wavefront reads 2*lines consecutive columns
// ---------------------------------------------------------------------------
template <typename T, int N, int BC, int PTM>
__global__ __launch_bounds__(PTM == 8 ? 512 : 256) void k_yfwd(T* __restrict__ data, int nx,
                                                               long plane, int llines,
                                                               const T* __restrict__ tab,
                                                               int nzm,
                                                               const int* __restrict__ skip) {
  using T2 = typename Vec2<T>::type;
  extern __shared__ unsigned char smem_raw[];
  if (skip && skip[blockIdx.y / nzm]) return;  // member already converged (whole block)
  const int lines = 1 << llines;
  const int q = threadIdx.x & (lines - 1), t = threadIdx.x >> llines;
  T2* col = reinterpret_cast<T2*>(data + (long)blockIdx.y * plane + (long)blockIdx.x * 2 * lines +
                                  2 * q);
  const int nx2 = nx >> 1;  // row stride in T2 units
  YLds<T, N> lds(reinterpret_cast<T2*>(smem_raw), q, lines);
  forward_body<T, N, BC, PTM>(
      lds, t, tab,
      [&](int e, T& r, T& i) {
        const T2 v = col[(long)e * nx2];
        r = v.x;
        i = v.y;
      },
      [&](int c0, T a0, T b0, int c1, T a1, T b1) {
        T2 v0, v1;
        v0.x = a0;
        v0.y = b0;
        v1.x = a1;
        v1.y = b1;
        col[(long)c0 * nx2] = v0;
        col[(long)c1 * nx2] = v1;
      });
}

template <typename T, int N, int BC, int PTM>
__global__ __launch_bounds__(PTM == 8 ? 512 : 256) void k_yinv(T* __restrict__ data, int nx,
                                                               long plane, int llines,
                                                               const T* __restrict__ tab,
                                                               int nzm,
                                                               const int* __restrict__ skip) {
  using T2 = typename Vec2<T>::type;
  extern __shared__ unsigned char smem_raw[];
  if (skip && skip[blockIdx.y / nzm]) return;  // member already converged (whole block)
  const int lines = 1 << llines;
  const int q = threadIdx.x & (lines - 1), t = threadIdx.x >> llines;
  T2* col = reinterpret_cast<T2*>(data + (long)blockIdx.y * plane + (long)blockIdx.x * 2 * lines +
                                  2 * q);
  const int nx2 = nx >> 1;
  YLds<T, N> lds(reinterpret_cast<T2*>(smem_raw), q, lines);
  inverse_body<T, N, BC, PTM>(
      lds, t, tab,
      [&](int c0, int c1, T& a0, T& b0, T& a1, T& b1) {
        const T2 v0 = col[(long)c0 * nx2], v1 = col[(long)c1 * nx2];
        a0 = v0.x;
        b0 = v0.y;
        a1 = v1.x;
        b1 = v1.y;
      },
      [&](int e, T r, T i) {
        T2 v;
        v.x = r;
        v.y = i;
        col[(long)e * nx2] = v;
      });
}

// ---------------------------------------------------------------------------
// quarter-wave x and y passes (BC_ND, BC_DN): one line per complex FFT of
// length N/2.  x: a block owns LPB consecutive rows, TPL threads each.  y:
// a block owns a tile of `cols` consecutive columns of one z-plane, thread
// (q, t) with q fastest.  The forward pass writes the DCT-IV coefficients in
// natural order; the inverse applies the same transform and doubles it, so
// that inverse(forward(x)) = N x as for the other transforms.  The x
// kernels take the same batch, shift, accumulation, skip and norm options as
// k_xfwd / k_xinv.
// ---------------------------------------------------------------------------
template <int N, int PTM>
constexpr int xq_rows_per_block() {
  return 256 / FftShape<N / 2, PTM>::TPL;
}

template <typename TI, typename T, int N, int BC, bool SUB, int PTM>
__global__ __launch_bounds__(256) void k_xqfwd(const Batch<const TI> in, T* __restrict__ out,
                                                long ostride, long nrows,
                                                const T* __restrict__ tab,
                                                const double* __restrict__ sub,
                                                const int* __restrict__ skip) {
  constexpr int H = N / 2, TPL = FftShape<H, PTM>::TPL, LPB = 256 / TPL;
  __shared__ T lds_mem[2 * LPB * lds_len<H>()];
  if (skip && skip[blockIdx.y]) return;  // member already converged (whole block)
  const int q = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long row = (long)blockIdx.x * LPB + q;
  const bool ok = row < nrows;
  const TI* g = in.p[blockIdx.y] + row * N;
  T* o = out + blockIdx.y * ostride + row * N;
  TI shift = TI(0);
  if constexpr (SUB) shift = TI(sub[blockIdx.y]);
  XLds<T, H> lds(lds_mem, q, LPB);
  quarter_body<T, N, PTM>(
      lds, t, tab,
      [&](int e, T& v) {
        if constexpr (SUB) v = ok ? T(g[qpos<N, BC>(e)] - shift) : T(0);
        else v = ok ? T(g[qpos<N, BC>(e)]) : T(0);
      },
      [&](int c, T v) {
        if (ok) o[c] = v;
      });
}

// block sums of e^2 and p^2 to norms[2 * (member * gridDim.x + block) + {0, 1}]
// (fixed order, through the block's LDS, which the caller no longer needs)
__device__ __forceinline__ void block_norms(double* red, double ee, double pp,
                                            double* __restrict__ norms) {
  __syncthreads();
  red[threadIdx.x] = ee;
  red[256 + threadIdx.x] = pp;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      red[256 + threadIdx.x] += red[256 + threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const long o = 2 * ((long)blockIdx.y * gridDim.x + blockIdx.x);
    norms[o] = red[0];
    norms[o + 1] = red[256];
  }
}

template <typename T, typename TO, int N, int BC, bool ACCUM, int PTM>
__global__ __launch_bounds__(256) void k_xqinv(const T* __restrict__ in, long istride,
                                                const Batch<TO> out, long nrows,
                                                const T* __restrict__ tab,
                                                const double* __restrict__ sub,
                                                const int* __restrict__ skip,
                                                double* __restrict__ norms) {
  constexpr int H = N / 2, TPL = FftShape<H, PTM>::TPL, LPB = 256 / TPL;
  constexpr bool NORMS = !std::is_same<T, TO>::value;
  // the norm reduction needs 512 doubles of LDS
  constexpr int LDS_T = 2 * LPB * lds_len<H>();
  constexpr int RED_T = 512 * (int)sizeof(double) / (int)sizeof(T);
  __shared__ T lds_mem[LDS_T > RED_T ? LDS_T : RED_T];
  if (skip && skip[blockIdx.y]) return;  // member already converged (whole block)
  double ee = 0.0, pp = 0.0;
  const int q = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long row = (long)blockIdx.x * LPB + q;
  const bool ok = row < nrows;
  const T* ia = in + blockIdx.y * istride + row * N;
  TO* o = out.p[blockIdx.y] + row * N;
  TO shift = TO(0);
  if constexpr (ACCUM) {
    if (sub) shift = TO(sub[blockIdx.y]);
  }
  XLds<T, H> lds(lds_mem, q, LPB);
  quarter_body<T, N, PTM>(
      lds, t, tab, [&](int c, T& v) { v = ok ? ia[c] : T(0); },
      [&](int e, T v) {
        if (!ok) return;
        const int p = qpos<N, BC>(e);
        const TO d = TO(T(2) * v) - shift;
        TO pv = d;
        if constexpr (ACCUM) pv = o[p] + d;
        o[p] = pv;
        if constexpr (NORMS) {
          ee += double(d) * double(d);
          pp += double(pv) * double(pv);
        }
      });
  if constexpr (NORMS) {
    if (norms) block_norms(reinterpret_cast<double*>(lds_mem), ee, pp, norms);
  }
}

template <typename T, int N, int BC, bool INV, int PTM>
__global__ __launch_bounds__(512) void k_yq(T* __restrict__ data, int nx, long plane, int lcols,
                                             const T* __restrict__ tab, int nzm,
                                             const int* __restrict__ skip) {
  using T2 = typename Vec2<T>::type;
  extern __shared__ unsigned char smem_raw[];
  if (skip && skip[blockIdx.y / nzm]) return;  // member already converged (whole block)
  const int cols = 1 << lcols;
  const int q = threadIdx.x & (cols - 1), t = threadIdx.x >> lcols;
  T* col = data + (long)blockIdx.y * plane + (long)blockIdx.x * cols + q;
  YLds<T, N / 2> lds(reinterpret_cast<T2*>(smem_raw), q, cols);
  if constexpr (INV) {
    quarter_body<T, N, PTM>(
        lds, t, tab, [&](int c, T& v) { v = col[(long)c * nx]; },
        [&](int e, T v) { col[(long)qpos<N, BC>(e) * nx] = T(2) * v; });
  } else {
    quarter_body<T, N, PTM>(
        lds, t, tab, [&](int e, T& v) { v = col[(long)qpos<N, BC>(e) * nx]; },
        [&](int c, T v) { col[(long)c * nx] = v; });
  }
}

// ---------------------------------------------------------------------------
// spectral z pass (uniform z): block (tile, member); tile = 2*lines
// consecutive (kx, ky) positions of the plane, each a z-line of N values
// `plane` apart.  Per packed z coefficient c of line (kx, ky):
//   x <- x * scale / (lamx[kx] + lamy[ky] + lamz[c]),  0 where that is 0
// (only the constant mode), which is the pseudo-inverse; the removed
// constant (the coefficient times scale: the mean) goes to mean_out[member].
// ---------------------------------------------------------------------------
template <typename T, int N, int BC, int PTM>
__global__ __launch_bounds__(PTM == 8 ? 512 : 256) void k_zspec(
    T* __restrict__ data, int nx, int lx, long plane, int llines, const T* __restrict__ tab,
    const double* __restrict__ lamx, const double* __restrict__ lamy,
    const double* __restrict__ lamz, double scale, long batch_stride,
    double* __restrict__ mean_out, const int* __restrict__ skip) {
  using T2 = typename Vec2<T>::type;
  extern __shared__ unsigned char smem_raw[];
  if (skip && skip[blockIdx.y]) return;  // member already converged (whole block)
  const int lines = 1 << llines;
  const int q = threadIdx.x & (lines - 1), t = threadIdx.x >> llines;
  const long pos = (long)blockIdx.x * 2 * lines + 2 * q;  // line a; line b = pos + 1
  T2* col = reinterpret_cast<T2*>(data + blockIdx.y * batch_stride + pos);
  const long pstride = plane >> 1;  // z stride in T2 units
  const double la = lamx[pos % nx] + lamy[pos / nx];
  const double lb = lamx[(pos + 1) % nx] + lamy[(pos + 1) / nx];
  YLds<T, N> lds(reinterpret_cast<T2*>(smem_raw), q, lines);
  spectral_body<T, N, BC, PTM>(
      lds, t, tab,
      [&](int e, T& r, T& i) {
        const T2 v = col[(long)e * pstride];
        r = v.x;
        i = v.y;
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
        T2 v;
        v.x = r;
        v.y = i;
        col[(long)e * pstride] = v;
      });
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
#define VP_SIZES(X) \
  X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(40) X(80) X(160) X(320) X(640)

// pt: values per thread of the radix schedule, 16 or 8 (a tuning knob; the
// results are the same up to rounding order)
template <int PTM>
static long x_rows_per_block(int n) {
  switch (n) {
#define VP_RPB(NN) \
  case NN: return 2L * (256 / FftShape<NN, PTM>::TPL);
    VP_SIZES(VP_RPB)
#undef VP_RPB
    default: return 0;
  }
}

template <int PTM>
static long xq_rows(int n) {
  switch (n) {
#define VP_RPB(NN) \
  case NN: return xq_rows_per_block<NN, PTM>();
    VP_SIZES(VP_RPB)
#undef VP_RPB
    default: return 0;
  }
}

long xpass_blocks(int nx, int bc, int pt, long nrows) {
  long rpb;
  if (bc == BC_ND || bc == BC_DN) rpb = pt == 8 ? xq_rows<8>(nx) : xq_rows<16>(nx);
  else rpb = pt == 8 ? x_rows_per_block<8>(nx) : x_rows_per_block<16>(nx);
  return rpb > 0 ? (nrows + rpb - 1) / rpb : 0;
}

template <typename TI, typename T, int BC, bool SUB, int PTM>
static hipError_t launch_xfwd_pt(const Batch<const TI>& in, int nb, T* out, long ostride, int n,
                                 long nrows, const T* tab, const PassOpts& o, hipStream_t st) {
#define VP_XF(NN)                                                                           \
  case NN: {                                                                                \
    const long rpb = 2 * (256 / FftShape<NN, PTM>::TPL);                                    \
    hipLaunchKernelGGL((k_xfwd<TI, T, NN, BC, SUB, PTM>),                                   \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb), dim3(256), 0, \
                       st, in, out, ostride, nrows, tab, o.sub, o.skip);                    \
    break;                                                                                  \
  }
  if (nb < 1 || nb > kMaxBatch) return hipErrorInvalidValue;
  switch (n) {
    VP_SIZES(VP_XF)
    default: return hipErrorInvalidValue;
  }
#undef VP_XF
  return hipGetLastError();
}

template <typename TI, typename T, int BC, bool SUB, int PTM>
static hipError_t launch_xqfwd_pt(const Batch<const TI>& in, int nb, T* out, long ostride, int n,
                                  long nrows, const T* tab, const PassOpts& o, hipStream_t st) {
#define VP_XQF(NN)                                                                          \
  case NN: {                                                                                \
    constexpr long rpb = xq_rows_per_block<NN, PTM>();                                      \
    hipLaunchKernelGGL((k_xqfwd<TI, T, NN, BC, SUB, PTM>),                                  \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb), dim3(256), 0, \
                       st, in, out, ostride, nrows, tab, o.sub, o.skip);                    \
    break;                                                                                  \
  }
  if (nb < 1 || nb > kMaxBatch) return hipErrorInvalidValue;
  switch (n) {
    VP_SIZES(VP_XQF)
    default: return hipErrorInvalidValue;
  }
#undef VP_XQF
  return hipGetLastError();
}

template <typename TI, typename T, int BC, bool SUB>
static hipError_t launch_xfwd_bc(const Batch<const TI>& in, int nb, T* out, long ostride, int n,
                                 long nrows, const T* tab, int pt, const PassOpts& o,
                                 hipStream_t st) {
  if constexpr (BC == BC_ND || BC == BC_DN)
    return pt == 8
               ? launch_xqfwd_pt<TI, T, BC, SUB, 8>(in, nb, out, ostride, n, nrows, tab, o, st)
               : launch_xqfwd_pt<TI, T, BC, SUB, 16>(in, nb, out, ostride, n, nrows, tab, o, st);
  else
    return pt == 8
               ? launch_xfwd_pt<TI, T, BC, SUB, 8>(in, nb, out, ostride, n, nrows, tab, o, st)
               : launch_xfwd_pt<TI, T, BC, SUB, 16>(in, nb, out, ostride, n, nrows, tab, o, st);
}

template <typename T, typename TO, int BC, bool ACCUM, int PTM>
static hipError_t launch_xinv_pt(const T* in, long istride, const Batch<TO>& out, int nb, int n,
                                 long nrows, const T* tab, const PassOpts& o, hipStream_t st) {
#define VP_XI(NN)                                                                           \
  case NN: {                                                                                \
    const long rpb = 2 * (256 / FftShape<NN, PTM>::TPL);                                    \
    hipLaunchKernelGGL((k_xinv<T, TO, NN, BC, ACCUM, PTM>),                                 \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb), dim3(256), 0, \
                       st, in, istride, out, nrows, tab, o.sub, o.skip, o.norms);           \
    break;                                                                                  \
  }
  if (nb < 1 || nb > kMaxBatch) return hipErrorInvalidValue;
  switch (n) {
    VP_SIZES(VP_XI)
    default: return hipErrorInvalidValue;
  }
#undef VP_XI
  return hipGetLastError();
}

template <typename T, typename TO, int BC, bool ACCUM, int PTM>
static hipError_t launch_xqinv_pt(const T* in, long istride, const Batch<TO>& out, int nb, int n,
                                  long nrows, const T* tab, const PassOpts& o, hipStream_t st) {
#define VP_XQI(NN)                                                                          \
  case NN: {                                                                                \
    constexpr long rpb = xq_rows_per_block<NN, PTM>();                                      \
    hipLaunchKernelGGL((k_xqinv<T, TO, NN, BC, ACCUM, PTM>),                                \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb), dim3(256), 0, \
                       st, in, istride, out, nrows, tab, o.sub, o.skip, o.norms);           \
    break;                                                                                  \
  }
  if (nb < 1 || nb > kMaxBatch) return hipErrorInvalidValue;
  switch (n) {
    VP_SIZES(VP_XQI)
    default: return hipErrorInvalidValue;
  }
#undef VP_XQI
  return hipGetLastError();
}

template <typename T, typename TO, int BC, bool ACCUM>
static hipError_t launch_xinv_bc(const T* in, long istride, const Batch<TO>& out, int nb, int n,
                                 long nrows, const T* tab, int pt, const PassOpts& o,
                                 hipStream_t st) {
  if constexpr (BC == BC_ND || BC == BC_DN)
    return pt == 8
               ? launch_xqinv_pt<T, TO, BC, ACCUM, 8>(in, istride, out, nb, n, nrows, tab, o, st)
               : launch_xqinv_pt<T, TO, BC, ACCUM, 16>(in, istride, out, nb, n, nrows, tab, o, st);
  else
    return pt == 8
               ? launch_xinv_pt<T, TO, BC, ACCUM, 8>(in, istride, out, nb, n, nrows, tab, o, st)
               : launch_xinv_pt<T, TO, BC, ACCUM, 16>(in, istride, out, nb, n, nrows, tab, o, st);
}

// y tile: `lines` column pairs per block (the radix-16 thread count of 256
// when the plane is wide enough, so both schedules read equally wide tiles);
// 2*lines columns divide nx (both powers of two)
// threads per line of the radix-16 schedule of length n (20 values per
// thread for lengths 5 * 2^k)
static int fft_tpl(int n) {
  if (n % 5 == 0) return n >= 20 ? n / 20 : 1;
  return n >= 16 ? n / 16 : 1;
}
// largest power of two dividing n
static long pow2_part(long n) { return n & -n; }

static int ypass_lines(int nx, int ny) {
  int lines = 256 / fft_tpl(ny);
  if (lines < 1) lines = 1;
  if (lines > pow2_part(nx) / 2) lines = (int)(pow2_part(nx) / 2);  // 2 lines divide nx
  return lines;
}

int ypass_tile_cols(int nx, int ny) { return 2 * ypass_lines(nx, ny); }

// quarter-wave y pass: one column per line, 2*lines columns per block
template <typename T, int BC, bool FWD, int PTM>
static hipError_t launch_yq_pt(T* data, int nx, int ny, int nplanes, const T* tab, int lines,
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
    auto kern = &k_yq<T, NN, BC, !FWD, PTM>;                                       \
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

template <typename T, int BC, bool FWD, int PTM>
static hipError_t launch_ystd_pt(T* data, int nx, int ny, int nplanes, const T* tab, int lines,
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
    auto kern = FWD ? &k_yfwd<T, NN, BC, PTM> : &k_yinv<T, NN, BC, PTM>;           \
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

template <typename T, int BC, bool FWD, int PTM>
static hipError_t launch_y_pt(T* data, int nx, int ny, int nplanes, const T* tab,
                              const PassOpts& o, hipStream_t st) {
  int lines = ypass_lines(nx, ny);
  if (o.lines > 0 && o.lines < lines) lines = o.lines;
  const int nzm = o.nzm > 0 ? o.nzm : nplanes;
  if constexpr (BC == BC_ND || BC == BC_DN)
    return launch_yq_pt<T, BC, FWD, PTM>(data, nx, ny, nplanes, tab, lines, nzm, o.skip, st);
  else
    return launch_ystd_pt<T, BC, FWD, PTM>(data, nx, ny, nplanes, tab, lines, nzm, o, st);
}

template <typename T, int BC, bool FWD>
static hipError_t launch_y_bc(T* data, int nx, int ny, int nplanes, const T* tab, int pt,
                              const PassOpts& o, hipStream_t st) {
  return pt == 8 ? launch_y_pt<T, BC, FWD, 8>(data, nx, ny, nplanes, tab, o, st)
                 : launch_y_pt<T, BC, FWD, 16>(data, nx, ny, nplanes, tab, o, st);
}

template <typename T, int BC, int PTM>
static hipError_t launch_zspec_pt(T* data, const ZSpecArgs& a, const T* tab, int nb,
                                  const int* skip, hipStream_t st) {
  using T2 = typename Vec2<T>::type;
  const long plane = (long)a.nx * a.ny;
  // tile width: as for the y pass of a line of the same length, or a.lines
  int lines = 256 / fft_tpl(a.nz);
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
    auto kern = &k_zspec<T, NN, BC, PTM>;                                                  \
    if (shm > 65536) {                                                                     \
      const hipError_t e = allow_large_lds(kern);                                          \
      if (e != hipSuccess) return e;                                                       \
    }                                                                                      \
    hipLaunchKernelGGL(kern, grid, dim3(nthr), shm, st, data, a.nx, a.lx, plane, ll, tab,  \
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

// calls f(std::integral_constant<int, BC>{}) for the run-time boundary code
template <typename F>
static hipError_t with_bc(int bc, F&& f) {
  switch (bc) {
    case BC_P: return f(std::integral_constant<int, BC_P>{});
    case BC_N: return f(std::integral_constant<int, BC_N>{});
    case BC_D: return f(std::integral_constant<int, BC_D>{});
    case BC_ND: return f(std::integral_constant<int, BC_ND>{});
    case BC_DN: return f(std::integral_constant<int, BC_DN>{});
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_zspec_t(T* data, const ZSpecArgs& a, const T* tab, int pt, int nb,
                                 const int* skip, hipStream_t st) {
  return with_bc(a.bcz, [&](auto B) -> hipError_t {
    constexpr int BC = decltype(B)::value;
    if constexpr (BC == BC_ND || BC == BC_DN)
      return hipErrorInvalidValue;  // the tridiagonal pass takes these
    else
      return pt == 8 ? launch_zspec_pt<T, BC, 8>(data, a, tab, nb, skip, st)
                     : launch_zspec_pt<T, BC, 16>(data, a, tab, nb, skip, st);
  });
}

hipError_t launch_zspec_f64(double* data, const ZSpecArgs& a, const double* tab, int pt, int nb,
                            hipStream_t st) {
  return launch_zspec_t<double>(data, a, tab, pt, nb, nullptr, st);
}
hipError_t launch_zspec_f32(float* data, const ZSpecArgs& a, const float* tab, int pt, int nb,
                            const int* skip, hipStream_t st) {
  return launch_zspec_t<float>(data, a, tab, pt, nb, skip, st);
}

hipError_t launch_xfwd_f64(const Batch<const double>& in, int nb, double* out, long ostride,
                           int nx, int bc, long nrows, const double* tab, int pt,
                           hipStream_t st) {
  const PassOpts o{};
  return with_bc(bc, [&](auto B) {
    return launch_xfwd_bc<double, double, decltype(B)::value, false>(in, nb, out, ostride, nx,
                                                                     nrows, tab, pt, o, st);
  });
}
hipError_t launch_xinv_f64(const double* in, long istride, const Batch<double>& out, int nb,
                           int nx, int bc, long nrows, const double* tab, int pt,
                           hipStream_t st) {
  const PassOpts o{};
  return with_bc(bc, [&](auto B) {
    return launch_xinv_bc<double, double, decltype(B)::value, false>(in, istride, out, nb, nx,
                                                                     nrows, tab, pt, o, st);
  });
}
hipError_t launch_xfwd_f32(const Batch<const double>& in, int nb, float* out, long ostride,
                           int nx, int bc, long nrows, const float* tab, int pt,
                           const PassOpts& o, hipStream_t st) {
  return with_bc(bc, [&](auto B) {
    constexpr int BC = decltype(B)::value;
    return o.sub ? launch_xfwd_bc<double, float, BC, true>(in, nb, out, ostride, nx, nrows, tab,
                                                           pt, o, st)
                 : launch_xfwd_bc<double, float, BC, false>(in, nb, out, ostride, nx, nrows, tab,
                                                            pt, o, st);
  });
}
hipError_t launch_xinv_f32(const float* in, long istride, const Batch<double>& out, int nb,
                           int nx, int bc, long nrows, bool accum, const float* tab, int pt,
                           const PassOpts& o, hipStream_t st) {
  return with_bc(bc, [&](auto B) {
    constexpr int BC = decltype(B)::value;
    return accum ? launch_xinv_bc<float, double, BC, true>(in, istride, out, nb, nx, nrows, tab,
                                                           pt, o, st)
                 : launch_xinv_bc<float, double, BC, false>(in, istride, out, nb, nx, nrows, tab,
                                                            pt, o, st);
  });
}
hipError_t launch_y_f64(double* data, int nx, int ny, int nplanes, int bc, bool fwd,
                        const double* tab, int pt, int lines, hipStream_t st) {
  PassOpts o{};
  o.lines = lines;
  return with_bc(bc, [&](auto B) {
    constexpr int BC = decltype(B)::value;
    return fwd ? launch_y_bc<double, BC, true>(data, nx, ny, nplanes, tab, pt, o, st)
               : launch_y_bc<double, BC, false>(data, nx, ny, nplanes, tab, pt, o, st);
  });
}
hipError_t launch_y_f32(float* data, int nx, int ny, int nplanes, int bc, bool fwd,
                        const float* tab, int pt, const PassOpts& o, hipStream_t st) {
  return with_bc(bc, [&](auto B) {
    constexpr int BC = decltype(B)::value;
    return fwd ? launch_y_bc<float, BC, true>(data, nx, ny, nplanes, tab, pt, o, st)
               : launch_y_bc<float, BC, false>(data, nx, ny, nplanes, tab, pt, o, st);
  });
}

}  // namespace vp
