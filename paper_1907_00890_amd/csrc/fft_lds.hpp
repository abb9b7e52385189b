// Radix-8/4/2 Stockham FFT on lines held in LDS, plus the pre/post steps that
// turn one complex transform into two real transforms (periodic: real DFT in
// packed form; walls: DCT-II / DCT-III by the even/odd reordering of
// J. Makhoul, "A fast cosine transform in one and two dimensions", IEEE
// TASSP 28(1), 1980).
//
// These transforms diagonalise the 1-D second difference of the staggered
// grid (the constant-coefficient Poisson operator of section 3.2) in x and y.
//
// Packed spectrum of one real line of length N (coefficient position c):
//   periodic:  c=0 -> Re X_0, c=1 -> Re X_{N/2}, c=2m -> Re X_m, c=2m+1 -> Im X_m
//              (X_m = sum_j x_j e^{-2 pi i j m / N}), eigenvalue index m
//   walls:     c=m -> X_m = sum_j x_j cos(pi m (2j+1) / (2N)), eigenvalue index m
// The inverse routines return N times the original line (no 1/N scaling).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace vp {

// ---------------------------------------------------------------------------
// small DFTs in registers; SIGN = -1 forward (e^{-i...}), +1 inverse
// ---------------------------------------------------------------------------
template <int SIGN, typename T>
__device__ __forceinline__ void mul_pm_i(T& r, T& i) {
  // (r + i I) * (SIGN I)
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
  T t1r = (orr[1] - T(SIGN) * oi[1]) * h, t1i = (T(SIGN) * orr[1] + oi[1]) * h;
  T t2r = orr[2], t2i = oi[2];
  mul_pm_i<SIGN>(t2r, t2i);
  T t3r = (-orr[3] - T(SIGN) * oi[3]) * h, t3i = (T(SIGN) * orr[3] - oi[3]) * h;
  r[0] = er[0] + orr[0]; i[0] = ei[0] + oi[0];
  r[4] = er[0] - orr[0]; i[4] = ei[0] - oi[0];
  r[1] = er[1] + t1r; i[1] = ei[1] + t1i;
  r[5] = er[1] - t1r; i[5] = ei[1] - t1i;
  r[2] = er[2] + t2r; i[2] = ei[2] + t2i;
  r[6] = er[2] - t2r; i[6] = ei[2] - t2i;
  r[3] = er[3] + t3r; i[3] = ei[3] + t3i;
  r[7] = er[3] - t3r; i[7] = ei[3] - t3i;
}

template <int R, int SIGN, typename T>
__device__ __forceinline__ void dftR(T* r, T* i) {
  if constexpr (R == 8) dft8<SIGN>(r, i);
  else if constexpr (R == 4) dft4<SIGN>(r, i);
  else dft2<SIGN>(r, i);
}

// even/odd reordering behind the DCT: FFT input position p holds x[perm(p)]
template <int N>
__device__ __forceinline__ int dct_perm(int p) {
  return p < N / 2 ? 2 * p : 2 * (N - 1 - p) + 1;
}

// ---------------------------------------------------------------------------
// Stockham passes.  Each of the TPL threads of a line performs (N/R)/TPL
// radix-R butterflies per pass; lines are read and written in place in LDS
// (element e of a line at re[e*es], im[e*es]) with a block barrier between the
// reads and the writes of every pass.  twc[k] = cos(2 pi k / N) and
// tws[k] = sin(2 pi k / N) for k in [0, N).
// PERM_IN permutes the reads of the first pass, PERM_OUT the writes of the
// last one (the DCT reordering and its inverse).
// ---------------------------------------------------------------------------
template <typename T, int N, int TPL, int SIGN, bool PERM_IN, bool PERM_OUT, int NS>
__device__ __forceinline__ void stockham(T* __restrict__ re, T* __restrict__ im, int es, int t,
                                         const T* __restrict__ twc, const T* __restrict__ tws) {
  constexpr int REM = N / NS;
  if constexpr (REM > 1) {
    constexpr int R = REM >= 8 ? 8 : REM;
    constexpr int NB = N / R;
    constexpr int BPT = NB / TPL;
    static_assert(BPT >= 1 && BPT * TPL == NB, "threads per line must divide N/R");
    constexpr bool FIRST = (NS == 1);
    constexpr bool LAST = (NS * R == N);
    T vr[BPT][R], vi[BPT][R];
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int j = t + TPL * b;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int src = j + r * NB;
        if constexpr (PERM_IN && FIRST) src = dct_perm<N>(src);
        vr[b][r] = re[src * es];
        vi[b][r] = im[src * es];
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int j = t + TPL * b;
      const int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const int ti = k * r * (N / (NS * R));
          const T wr = twc[ti], wi = T(SIGN) * tws[ti];
          const T xr = vr[b][r], xi = vi[b][r];
          vr[b][r] = xr * wr - xi * wi;
          vi[b][r] = xr * wi + xi * wr;
        }
      }
      dftR<R, SIGN>(vr[b], vi[b]);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int dst = base + r * NS;
        if constexpr (PERM_OUT && LAST) dst = dct_perm<N>(dst);
        re[dst * es] = vr[b][r];
        im[dst * es] = vi[b][r];
      }
    }
    __syncthreads();
    stockham<T, N, TPL, SIGN, PERM_IN, PERM_OUT, NS * R>(re, im, es, t, twc, tws);
  }
}

// ---------------------------------------------------------------------------
// Forward: two real lines a, b -> their packed spectra (in place).
// The caller has stored a in the "re" slots and b in the "im" slots; on
// return the re slots hold a's packed spectrum and the im slots b's.
// pc[m] = cos(pi m / (2N)), ps[m] = sin(pi m / (2N)) for m in [0, N/2].
// ---------------------------------------------------------------------------
template <typename T, int N, int BC, int TPL>
__device__ __forceinline__ void real_pair_forward(T* __restrict__ a, T* __restrict__ b, int es, int t,
                                                  const T* __restrict__ twc, const T* __restrict__ tws,
                                                  const T* __restrict__ pc, const T* __restrict__ ps) {
  stockham<T, N, TPL, -1, BC == BC_N, false, 1>(a, b, es, t, twc, tws);
  constexpr int MPT = (N / 2) / TPL;  // modes per thread, m in [0, N/2)
  static_assert(MPT * TPL == N / 2, "bad TPL");
  T zr[MPT], zi[MPT], wr[MPT], wi[MPT];
  T hr = T(0), hi = T(0);  // Z[N/2], read by thread 0
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int m = t + TPL * u;
    const int mm = (N - m) & (N - 1);
    zr[u] = a[m * es]; zi[u] = b[m * es];
    wr[u] = a[mm * es]; wi[u] = b[mm * es];
  }
  if (t == 0) { hr = a[(N / 2) * es]; hi = b[(N / 2) * es]; }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int m = t + TPL * u;
    // A = (Z_m + conj Z_{N-m}) / 2,  B = (Z_m - conj Z_{N-m}) / (2i)
    const T Ar = T(0.5) * (zr[u] + wr[u]), Ai = T(0.5) * (zi[u] - wi[u]);
    const T Br = T(0.5) * (zi[u] + wi[u]), Bi = T(0.5) * (wr[u] - zr[u]);
    if constexpr (BC == BC_P) {
      if (m == 0) {
        a[0] = zr[u]; b[0] = zi[u];
        a[es] = hr; b[es] = hi;
      } else {
        a[(2 * m) * es] = Ar; a[(2 * m + 1) * es] = Ai;
        b[(2 * m) * es] = Br; b[(2 * m + 1) * es] = Bi;
      }
    } else {
      if (m == 0) {
        const T h = T(0.70710678118654752440084436210485);
        a[0] = zr[u]; b[0] = zi[u];
        a[(N / 2) * es] = h * hr; b[(N / 2) * es] = h * hi;
      } else {
        // Y = e^{-i pi m/(2N)} V_m;  X_m = Re Y, X_{N-m} = -Im Y
        const T c = pc[m], s = ps[m];
        const T yAr = c * Ar + s * Ai, yAi = c * Ai - s * Ar;
        const T yBr = c * Br + s * Bi, yBi = c * Bi - s * Br;
        a[m * es] = yAr; a[(N - m) * es] = -yAi;
        b[m * es] = yBr; b[(N - m) * es] = -yBi;
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Inverse: two packed spectra (re slots: line a, im slots: line b) -> N times
// the two real lines, in place.
// ---------------------------------------------------------------------------
template <typename T, int N, int BC, int TPL>
__device__ __forceinline__ void real_pair_inverse(T* __restrict__ a, T* __restrict__ b, int es, int t,
                                                  const T* __restrict__ twc, const T* __restrict__ tws,
                                                  const T* __restrict__ pc, const T* __restrict__ ps) {
  constexpr int MPT = (N / 2) / TPL;
  T z0r[MPT], z0i[MPT], z1r[MPT], z1i[MPT];
  T hr = T(0), hi = T(0);
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int m = t + TPL * u;
    if constexpr (BC == BC_P) {
      if (m == 0) {
        z0r[u] = a[0]; z0i[u] = b[0];
        hr = a[es]; hi = b[es];
        z1r[u] = T(0); z1i[u] = T(0);
      } else {
        const T Ar = a[(2 * m) * es], Ai = a[(2 * m + 1) * es];
        const T Br = b[(2 * m) * es], Bi = b[(2 * m + 1) * es];
        z0r[u] = Ar - Bi; z0i[u] = Ai + Br;   // Z_m = A + iB
        z1r[u] = Ar + Bi; z1i[u] = Br - Ai;   // Z_{N-m} = conj A + i conj B
      }
    } else {
      if (m == 0) {
        const T r2 = T(1.4142135623730950488016887242097);
        z0r[u] = a[0]; z0i[u] = b[0];
        hr = r2 * a[(N / 2) * es]; hi = r2 * b[(N / 2) * es];
        z1r[u] = T(0); z1i[u] = T(0);
      } else {
        // V_m = e^{+i pi m/(2N)} (X_m - i X_{N-m})
        const T c = pc[m], s = ps[m];
        const T xa = a[m * es], xan = a[(N - m) * es];
        const T xb = b[m * es], xbn = b[(N - m) * es];
        const T vAr = c * xa + s * xan, vAi = s * xa - c * xan;
        const T vBr = c * xb + s * xbn, vBi = s * xb - c * xbn;
        z0r[u] = vAr - vBi; z0i[u] = vAi + vBr;
        z1r[u] = vAr + vBi; z1i[u] = vBr - vAi;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int m = t + TPL * u;
    a[m * es] = z0r[u]; b[m * es] = z0i[u];
    if (m == 0) {
      a[(N / 2) * es] = hr; b[(N / 2) * es] = hi;
    } else {
      a[(N - m) * es] = z1r[u]; b[(N - m) * es] = z1i[u];
    }
  }
  __syncthreads();
  stockham<T, N, TPL, +1, false, BC == BC_N, 1>(a, b, es, t, twc, tws);
}

}  // namespace vp
