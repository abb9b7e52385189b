// Building blocks of the x, y and spectral z passes (transforms_x.hip,
// transforms_y.hip, transforms_z.hip): LDS access policies, the Stockham
// passes through LDS and the forward / inverse / spectral / quarter-wave
// bodies, shared by every pass.
//
// The passes are real-to-real transforms of
// every x-line (contiguous rows) and every y-line (columns of a z-plane), two
// real lines per complex FFT (see fft_lds.hpp for the packed spectra).
//
// Data path of a forward pass: the first Stockham pass loads straight from
// HBM into registers (a line's N/16 threads read consecutive addresses), the
// intermediate passes exchange through LDS, and the real-pair step reads the
// last pass from LDS and writes the packed spectrum straight to HBM.  The
// inverse mirrors it: the real-pair step loads from HBM into LDS and the last
// Stockham pass stores to HBM.  The cosine and sine transforms of x rows
// instead take one more LDS round trip for their even/odd reordering, so that
// rows are still read and written in element order.  One block owns 2*LPB
// whole rows (x) or a tile of 2*LINES columns of one z-plane (y), so every
// HBM access is a contiguous chunk.  LDS rows are padded by one slot every
// 16 values, which spreads the strided writes of the first pass over the
// banks.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_lds.hpp"
#include "kernels.hpp"

// The build compiles each transform source as several objects, one per part
// of its entry points (VP_PART = 1, 2, ...), so that the template
// instantiations of one file spread over parallel compiler jobs; without
// VP_PART one object holds every entry point.
#ifndef VP_PART
#define VP_PART 0
#endif
#define VP_IN_PART(k) (VP_PART == 0 || VP_PART == (k))

namespace vp {

__device__ __forceinline__ int lds_pos(int e) { return e + (e >> 4); }

template <int N>
constexpr int lds_len() {
  return N + N / 16 + 1;
}

// threads of an x-pass block: 256, or 128 for lengths 5 * 2^k (20 values per
// thread: a 256-thread block would hold about 88 KB of LDS, one block per CU)
template <int N>
constexpr int x_block_threads() {
  return odd_factor(N) == 5 ? 128 : 256;
}

// The radix knob (PTM 16 or 8) does not change the schedule of a length with
// an odd factor: both knob values launch the one PTM = 16 instantiation.
template <int N, int PTM>
constexpr int canon_ptm() {
  return odd_factor(N) > 1 ? 16 : PTM;
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
// c0 and c1 of both lines.  ROW (x passes, contiguous lines): the cosine and
// sine transforms load the line in element order and reorder it through LDS
// (the even/odd reordering read straight from HBM would take every other
// element of a row per load); y lines (ROW false) reorder whole rows of a
// tile, which stay contiguous, and load straight into the first pass.
// ---------------------------------------------------------------------------
template <typename T, int N, int BC, int PTM, bool ROW = false, typename L, typename Load,
          typename Store>
__device__ __forceinline__ void forward_body(L& lds, int t, const T* __restrict__ tab, Load load,
                                             Store store) {
  using S = FftShape<N, PTM>;
  constexpr int PT = S::PT, TPL = S::TPL;
  constexpr int R1 = PassRadix<N, 1, PTM>::R;
  T vr[PT], vi[PT];
  if constexpr (ROW && BC != BC_P) {
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int j = t + TPL * k;
      T re, im;
      load(j, re, im);
      if constexpr (BC == BC_D) flip_odd(j, re, im);
      lds.put(dct_unperm<N>(j), re, im);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PT; ++r) lds.get(pass_in<N, 1, PTM>(t, r / R1, r % R1), vr[r], vi[r]);
    __syncthreads();  // the first pass writes back over these positions
  } else {
#pragma unroll
    for (int r = 0; r < PT; ++r) {
      // inputs of the first pass's butterflies (t + r TPL when a thread holds one)
      int e = pass_in<N, 1, PTM>(t, r / R1, r % R1);
      if constexpr (BC != BC_P) e = dct_perm<N>(e);
      load(e, vr[r], vi[r]);
      if constexpr (BC == BC_D) flip_odd(e, vr[r], vi[r]);
    }
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
// and c1 of both lines; `store(e, re, im)` writes element e of lines a and b.
// ROW: as for forward_body, the cosine and sine inverses of x lines undo the
// even/odd reordering through LDS and store the line in element order.
template <typename T, int N, int BC, int PTM, bool ROW = false, typename L, typename Load2,
          typename Store>
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
  if constexpr (ROW && BC != BC_P) {
    later_passes<T, N, 1, +1, false, PTM>(lds, t, tab, vr, vi);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int j = t + TPL * k;
      T re, im;
      lds.get(dct_unperm<N>(j), re, im);
      if constexpr (BC == BC_D) flip_odd(j, re, im);
      store(j, re, im);
    }
    return;
  }
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
  return x_block_threads<N>() / FftShape<N / 2, PTM>::TPL;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
#define VP_SIZES(X)                                                                      \
  X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(40) X(80) X(160) X(320) X(640) X(24) \
      X(48) X(96) X(192) X(384) X(768)

// y tile: `lines` column pairs per block (the radix-16 thread count of 256
// when the plane is wide enough, so both schedules read equally wide tiles);
// 2*lines columns divide nx (both powers of two)
// threads of a y-pass or spectral z-pass block at the default tile width
// (128 for lengths 5 * 2^k: 20 values per thread, LDS per block)
static inline int pass_threads(int n) { return odd_factor(n) == 5 ? 128 : 256; }

// threads per line of the radix-16 schedule of length n (4F values per
// thread for lengths F * 2^k, F = 3, 5)
static inline int fft_tpl(int n) {
  const int f = odd_factor(n);
  if (f > 1) return n >= 4 * f ? n / (4 * f) : 1;
  return n >= 16 ? n / 16 : 1;
}

// largest power of two dividing n
static inline long pow2_part(long n) { return n & -n; }

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

}  // namespace vp
