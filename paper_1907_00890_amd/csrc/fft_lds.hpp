// Building blocks of the x and y transforms of the spectral Poisson solve
// (the constant-coefficient direct solver of section 3.2 diagonalises the
// 1-D second difference of the staggered grid in x and y).
//
// * Small DFTs in registers (radix 2, 3, 4, 5, 8, 16; radix 16 as 4 x 4).
// * Stockham passes of radix 16 first, then the remainder (plan<N>):
//   N = 256 -> 16 x 16, 512 -> 16 x 16 x 2, 1024 -> 16 x 16 x 4.  Each of the
//   N/16 threads of a line holds 16 complex values; pass p reads positions
//   j + r N/R and writes (j / NS) NS R + j % NS + r NS (NS = product of the
//   earlier radices).  Lengths F * 2^k with an odd factor F = 3 or 5: 4F
//   values per thread (so the threads of a line stay a power of two), a
//   radix-F pass, then radix 4 (and a last radix 2): 320 -> 5 x 4 x 4 x 4,
//   640 -> 5 x 4 x 4 x 4 x 2, 384 -> 3 x 4 x 4 x 4 x 2, 768 -> 3 x 4 x 4 x 4 x 4.
// * Two real lines per complex transform.  Periodic lines use a real DFT in
//   packed form, wall lines a DCT-II / DCT-III computed through the even/odd
//   reordering of J. Makhoul ("A fast cosine transform in one and two
//   dimensions", IEEE TASSP 28(1), 1980).  Packed spectrum of a real line of
//   length N, coefficient position c:
//     periodic: c=0 Re X_0, c=1 Re X_{N/2}, c=2m Re X_m, c=2m+1 Im X_m
//               (X_m = sum_j x_j e^{-2 pi i j m / N}), eigenvalue index m;
//     walls:    c=m X_m = sum_j x_j cos(pi m (2j+1) / (2N)), eigenvalue index m.
//   Inverse transforms return N times the line (no 1/N).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace vp {

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// ---------------------------------------------------------------------------
// small DFTs in registers; SIGN = -1 forward (e^{-i...}), +1 inverse
// ---------------------------------------------------------------------------
template <int SIGN, typename T>
__device__ __forceinline__ void mul_pm_i(T& r, T& i) {  // (r + i I) * (SIGN I)
  const T tr = r;
  if constexpr (SIGN < 0) { r = i; i = -tr; }
  else { r = -i; i = tr; }
}

template <int SIGN, typename T>
__device__ __forceinline__ void dft2(T* r, T* i) {
  const T tr = r[0] - r[1], ti = i[0] - i[1];
  r[0] += r[1]; i[0] += i[1];
  r[1] = tr; i[1] = ti;
}

template <int SIGN, typename T>
__device__ __forceinline__ void dft4(T* r, T* i) {
  const T a0r = r[0] + r[2], a0i = i[0] + i[2];
  const T a1r = r[0] - r[2], a1i = i[0] - i[2];
  const T a2r = r[1] + r[3], a2i = i[1] + i[3];
  T a3r = r[1] - r[3], a3i = i[1] - i[3];
  mul_pm_i<SIGN>(a3r, a3i);
  r[0] = a0r + a2r; i[0] = a0i + a2i;
  r[2] = a0r - a2r; i[2] = a0i - a2i;
  r[1] = a1r + a3r; i[1] = a1i + a3i;
  r[3] = a1r - a3r; i[3] = a1i - a3i;
}

template <int SIGN, typename T>
__device__ __forceinline__ void dft8(T* r, T* i) {
  T er[4] = {r[0], r[2], r[4], r[6]}, ei[4] = {i[0], i[2], i[4], i[6]};
  T orr[4] = {r[1], r[3], r[5], r[7]}, oi[4] = {i[1], i[3], i[5], i[7]};
  dft4<SIGN>(er, ei);
  dft4<SIGN>(orr, oi);
  const T h = T(0.70710678118654752440084436210485);
  // w^1 = (1 + SIGN i)/sqrt2, w^2 = SIGN i, w^3 = (-1 + SIGN i)/sqrt2
  const T t1r = (orr[1] - T(SIGN) * oi[1]) * h, t1i = (T(SIGN) * orr[1] + oi[1]) * h;
  T t2r = orr[2], t2i = oi[2];
  mul_pm_i<SIGN>(t2r, t2i);
  const T t3r = (-orr[3] - T(SIGN) * oi[3]) * h, t3i = (T(SIGN) * orr[3] - oi[3]) * h;
  r[0] = er[0] + orr[0]; i[0] = ei[0] + oi[0];
  r[4] = er[0] - orr[0]; i[4] = ei[0] - oi[0];
  r[1] = er[1] + t1r; i[1] = ei[1] + t1i;
  r[5] = er[1] - t1r; i[5] = ei[1] - t1i;
  r[2] = er[2] + t2r; i[2] = ei[2] + t2i;
  r[6] = er[2] - t2r; i[6] = ei[2] - t2i;
  r[3] = er[3] + t3r; i[3] = ei[3] + t3i;
  r[7] = er[3] - t3r; i[7] = ei[3] - t3i;
}

// radix 3: with a = x1 + x2, b = x1 - x2,
//   X0 = x0 + a,  X1, X2 = x0 - a/2 +- SIGN i (sqrt3/2) b
template <int SIGN, typename T>
__device__ __forceinline__ void dft3(T* r, T* i) {
  const T h = T(0.86602540378443864676372317075293618347);  // sqrt(3)/2
  const T ar = r[1] + r[2], ai = i[1] + i[2];
  const T ur = T(SIGN) * h * (r[1] - r[2]), ui = T(SIGN) * h * (i[1] - i[2]);
  const T tr = r[0] - T(0.5) * ar, ti = i[0] - T(0.5) * ai;
  r[0] = r[0] + ar;
  i[0] = i[0] + ai;
  r[1] = tr - ui; i[1] = ti + ur;  // t + i u
  r[2] = tr + ui; i[2] = ti - ur;  // t - i u
}

// radix 5: with a_1 = x1 + x4, b_1 = x1 - x4, a_2 = x2 + x3, b_2 = x2 - x3,
//   X0 = x0 + a_1 + a_2,
//   X1, X4 = x0 + c1 a_1 + c2 a_2 +- SIGN i (s1 b_1 + s2 b_2),
//   X2, X3 = x0 + c2 a_1 + c1 a_2 +- SIGN i (s2 b_1 - s1 b_2),
// c_m = cos(2 pi m/5), s_m = sin(2 pi m/5)
template <int SIGN, typename T>
__device__ __forceinline__ void dft5(T* r, T* i) {
  const T c1 = T(0.30901699437494742410229341718281905886);   // (sqrt5 - 1)/4
  const T c2 = T(-0.80901699437494742410229341718281905886);  // -(sqrt5 + 1)/4
  const T s1 = T(0.95105651629515357211643933337938214340);
  const T s2 = T(0.58778525229247312916870595463907276860);
  const T a1r = r[1] + r[4], a1i = i[1] + i[4], b1r = r[1] - r[4], b1i = i[1] - i[4];
  const T a2r = r[2] + r[3], a2i = i[2] + i[3], b2r = r[2] - r[3], b2i = i[2] - i[3];
  const T t1r = r[0] + c1 * a1r + c2 * a2r, t1i = i[0] + c1 * a1i + c2 * a2i;
  const T t2r = r[0] + c2 * a1r + c1 * a2r, t2i = i[0] + c2 * a1i + c1 * a2i;
  const T u1r = T(SIGN) * (s1 * b1r + s2 * b2r), u1i = T(SIGN) * (s1 * b1i + s2 * b2i);
  const T u2r = T(SIGN) * (s2 * b1r - s1 * b2r), u2i = T(SIGN) * (s2 * b1i - s1 * b2i);
  r[0] = r[0] + a1r + a2r;
  i[0] = i[0] + a1i + a2i;
  r[1] = t1r - u1i; i[1] = t1i + u1r;  // t + i u
  r[4] = t1r + u1i; i[4] = t1i - u1r;  // t - i u
  r[2] = t2r - u2i; i[2] = t2i + u2r;
  r[3] = t2r + u2i; i[3] = t2i - u2r;
}

// radix 16 as 4 x 4: DFT4 over n1 of x[4 n1 + n2] (index k1), twiddle
// w16^{n2 k1}, DFT4 over n2; output X[k1 + 4 k2]
template <int SIGN, typename T>
__device__ __forceinline__ void dft16(T* r, T* i) {
  T yr[4][4], yi[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
      yr[n2][n1] = r[4 * n1 + n2];
      yi[n2][n1] = i[4 * n1 + n2];
    }
    dft4<SIGN>(yr[n2], yi[n2]);
  }
  const T c1 = T(0.92387953251128675612818318939678828682);   // cos(pi/8)
  const T s1 = T(0.38268343236508977172845998403039886676);   // sin(pi/8)
  const T h = T(0.70710678118654752440084436210484903928);    // cos(pi/4)
  // w16^m = cos(2 pi m/16) + SIGN i sin(2 pi m/16) for m = n2 k1 in 1..9
  const T wc[10] = {T(1), c1, h, s1, T(0), -s1, -h, -c1, T(-1), -c1};
  const T ws[10] = {T(0), s1, h, c1, T(1), c1, h, s1, T(0), -s1};
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2) {
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) {
      const int m = n2 * k1;
      const T c = wc[m], s = T(SIGN) * ws[m];
      const T xr = yr[n2][k1], xi = yi[n2][k1];
      yr[n2][k1] = xr * c - xi * s;
      yi[n2][k1] = xr * s + xi * c;
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    T zr[4] = {yr[0][k1], yr[1][k1], yr[2][k1], yr[3][k1]};
    T zi[4] = {yi[0][k1], yi[1][k1], yi[2][k1], yi[3][k1]};
    dft4<SIGN>(zr, zi);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      r[k1 + 4 * k2] = zr[k2];
      i[k1 + 4 * k2] = zi[k2];
    }
  }
}

template <int R, int SIGN, typename T>
__device__ __forceinline__ void dftR(T* r, T* i) {
  if constexpr (R == 16) dft16<SIGN>(r, i);
  else if constexpr (R == 8) dft8<SIGN>(r, i);
  else if constexpr (R == 5) dft5<SIGN>(r, i);
  else if constexpr (R == 4) dft4<SIGN>(r, i);
  else if constexpr (R == 3) dft3<SIGN>(r, i);
  else dft2<SIGN>(r, i);
}

// even/odd reordering behind the DCT: FFT input position p holds x[perm(p)]
template <int N>
__device__ __forceinline__ int dct_perm(int p) {
  return p < N / 2 ? 2 * p : 2 * (N - 1 - p) + 1;
}
// its inverse: the FFT input position that holds element j
template <int N>
__device__ __forceinline__ int dct_unperm(int j) {
  return (j & 1) ? N - 1 - (j >> 1) : (j >> 1);
}

// ---------------------------------------------------------------------------
// pass bookkeeping
// ---------------------------------------------------------------------------
// PTM: complex values per thread (16: radix-16 passes, 8: radix-8 passes;
// the radix schedule of a length is greedy, largest radix first).  Lengths
// F * 2^k (F = 3, 5) take 4F values per thread whatever PTM (radix F, then 4,
// then 2).
__host__ __device__ constexpr int odd_factor(int n) {
  return n % 3 == 0 ? 3 : (n % 5 == 0 ? 5 : 1);
}
template <int N, int PTM = 16>
struct FftShape {
  static constexpr int F = odd_factor(N);
  static constexpr int PT = F > 1 ? (N >= 4 * F ? 4 * F : N)  // values per thread
                                  : (N >= PTM ? PTM : N);
  static constexpr int TPL = N / PT;  // threads per line
};
template <int N, int NS, int PTM = 16>
struct PassRadix {
  static constexpr int REM = N / NS;
  static constexpr int F = odd_factor(N);
  static constexpr int R = F > 1 ? (NS == 1 ? F : (REM >= 4 ? 4 : REM))
                                 : (REM >= PTM ? PTM : REM);
};

// Twiddles of one pass for this thread: w_N^{(j % NS) r N/(NS R)}, r = 1..R-1,
// for each of its PT/R butterflies j = t + TPL b.  tab holds the pairs
// (cos, sin)(2 pi k/N) at [2k], [2k + 1].
template <typename T, int N, int NS, int SIGN, int PTM>
__device__ __forceinline__ void load_twiddles(const T* __restrict__ tab, int t, T* wr, T* wi) {
  constexpr int R = PassRadix<N, NS, PTM>::R;
  constexpr int PT = FftShape<N, PTM>::PT, TPL = FftShape<N, PTM>::TPL;
  constexpr int B = PT / R;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int k = (t + TPL * b) % NS;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const int ti = k * r * (N / (NS * R));
      const typename Vec2<T>::type w = reinterpret_cast<const typename Vec2<T>::type*>(tab)[ti];
      wr[b * R + r] = w.x;
      wi[b * R + r] = T(SIGN) * w.y;
    }
  }
}

// twiddle + DFT of the thread's PT/R butterflies of one pass
template <typename T, int N, int NS, int SIGN, int PTM>
__device__ __forceinline__ void pass_compute(T* vr, T* vi, const T* wr, const T* wi) {
  constexpr int R = PassRadix<N, NS, PTM>::R;
  constexpr int B = FftShape<N, PTM>::PT / R;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const T xr = vr[b * R + r], xi = vi[b * R + r];
        const T c = wr[b * R + r], s = wi[b * R + r];
        vr[b * R + r] = xr * c - xi * s;
        vi[b * R + r] = xr * s + xi * c;
      }
    }
    dftR<R, SIGN>(vr + b * R, vi + b * R);
  }
}

// input position of value (b, r) of a pass, and output position
template <int N, int NS, int PTM>
__device__ __forceinline__ int pass_in(int t, int b, int r) {
  constexpr int R = PassRadix<N, NS, PTM>::R;
  return t + FftShape<N, PTM>::TPL * b + r * (N / R);
}
template <int N, int NS, int PTM>
__device__ __forceinline__ int pass_out(int t, int b, int r) {
  constexpr int R = PassRadix<N, NS, PTM>::R;
  const int j = t + FftShape<N, PTM>::TPL * b;
  return (j / NS) * NS * R + (j % NS) + r * NS;
}

// ---------------------------------------------------------------------------
// two real lines <-> one complex line: per-mode pre/post steps.
// For mode m in [1, N/2) the two spectra A_m, B_m of the real lines a, b
// follow from Z_m and Z_{N-m} of Z = FFT(a + i b):
//   A = (Z_m + conj Z_{N-m}) / 2,  B = (Z_m - conj Z_{N-m}) / (2i).
// c = cos(pi m/(2N)), s = sin(pi m/(2N)) (the DCT rotation).
// ---------------------------------------------------------------------------
template <typename T, int N, int BC>
struct RealPair {
  // forward: Z_m, Z_{N-m} -> outputs: periodic (a[2m], a[2m+1], b[2m], b[2m+1]);
  // walls (a[m], a[N-m], b[m], b[N-m])
  static __device__ __forceinline__ void post(T zr, T zi, T wr, T wi, T c, T s, T* oa, T* ob) {
    const T Ar = T(0.5) * (zr + wr), Ai = T(0.5) * (zi - wi);
    const T Br = T(0.5) * (zi + wi), Bi = T(0.5) * (wr - zr);
    if constexpr (BC == BC_P) {
      oa[0] = Ar; oa[1] = Ai;
      ob[0] = Br; ob[1] = Bi;
    } else {
      // Y = e^{-i pi m/(2N)} V_m;  X_m = Re Y, X_{N-m} = -Im Y
      oa[0] = c * Ar + s * Ai; oa[1] = -(c * Ai - s * Ar);
      ob[0] = c * Br + s * Bi; ob[1] = -(c * Bi - s * Br);
    }
  }
  // inverse: packed inputs of mode m -> Z_m, Z_{N-m}
  static __device__ __forceinline__ void pre(const T* ia, const T* ib, T c, T s, T& z0r, T& z0i,
                                             T& z1r, T& z1i) {
    if constexpr (BC == BC_P) {
      const T Ar = ia[0], Ai = ia[1], Br = ib[0], Bi = ib[1];
      z0r = Ar - Bi; z0i = Ai + Br;   // A + iB
      z1r = Ar + Bi; z1i = Br - Ai;   // conj A + i conj B
    } else {
      // V_m = e^{+i pi m/(2N)} (X_m - i X_{N-m}); ia = (X_m, X_{N-m})
      const T vAr = c * ia[0] + s * ia[1], vAi = s * ia[0] - c * ia[1];
      const T vBr = c * ib[0] + s * ib[1], vBi = s * ib[0] - c * ib[1];
      z0r = vAr - vBi; z0i = vAi + vBr;
      z1r = vAr + vBi; z1i = vBr - vAi;
    }
  }
};

}  // namespace vp
