// x passes of the spectral Poisson solve: every x-line (contiguous rows),
// two real lines per complex FFT (real DFT, DCT, sign-alternated DST), or
// one line per half-length FFT (quarter-wave DCT-IV), with the batch,
// shift, accumulation, skip and norm options of the mixed chain.
#include "transform_passes.hpp"

namespace vp {

// block sums of e^2 and p^2 to norms[2 * (member * gridDim.x + block) + {0, 1}]
// (fixed order, through the block's LDS, which the caller no longer needs;
// XB threads, red holds 2 XB doubles)
template <int XB>
__device__ __forceinline__ void block_norms(double* red, double ee, double pp,
                                            double* __restrict__ norms) {
  __syncthreads();
  red[threadIdx.x] = ee;
  red[XB + threadIdx.x] = pp;
  __syncthreads();
  for (int w = XB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      red[XB + threadIdx.x] += red[XB + threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const long o = 2 * ((long)blockIdx.y * gridDim.x + blockIdx.x);
    norms[o] = red[0];
    norms[o + 1] = red[XB];
  }
}

// ---------------------------------------------------------------------------
// x kernels: a block owns 2*LPB consecutive rows (nrows is even);
// x_block_threads<N>() threads, TPL per line pair
// ---------------------------------------------------------------------------
// SUB: member b's input is read as in[b] - sub[b] (FP64, before any
// conversion to T); without it the kernel reads its input unchanged.
template <typename TI, typename T, int N, int BC, bool SUB, int PTM>
__global__ __launch_bounds__(256) void k_xfwd(const Batch<const TI> in, T* __restrict__ out,
                                               long ostride, long nrows,
                                               const T* __restrict__ tab,
                                               const double* __restrict__ sub,
                                               const int* __restrict__ skip) {
  constexpr int TPL = FftShape<N, PTM>::TPL, LPB = x_block_threads<N>() / TPL;
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
  forward_body<T, N, BC, PTM, true>(
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
  constexpr int XB = x_block_threads<N>(), TPL = FftShape<N, PTM>::TPL, LPB = XB / TPL;
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
  inverse_body<T, N, BC, PTM, true>(
      lds, t, tab,
      [&](int c0, int c1, T& a0, T& b0, T& a1, T& b1) {
        if constexpr (BC == BC_P) {
          // the packed real DFT pairs positions c0 (even) and c1 = c0 + 1:
          // one vector load per row
          using T2 = typename Vec2<T>::type;
          T2 va{T(0), T(0)}, vb{T(0), T(0)};
          if (ok) {
            va = *reinterpret_cast<const T2*>(ia + c0);
            vb = *reinterpret_cast<const T2*>(ib + c0);
          }
          a0 = va.x;
          a1 = va.y;
          b0 = vb.x;
          b1 = vb.y;
        } else {
          a0 = ok ? ia[c0] : T(0);
          b0 = ok ? ib[c0] : T(0);
          a1 = ok ? ia[c1] : T(0);
          b1 = ok ? ib[c1] : T(0);
        }
      },
      [&](int e, T r, T i) {
        if (!ok) return;
        const TO da = TO(r) - shift, db = TO(i) - shift;
        TO pa = da, pb = db;
        if constexpr (ACCUM) {
          pa = oa[e] + da;
          pb = ob[e] + db;
        }
        // rows are stored in element order, non-temporally (the result is
        // not read again by this pass; measured at 256^3, two fields per
        // launch: 107 -> 86 us)
        __builtin_nontemporal_store(pa, oa + e);
        __builtin_nontemporal_store(pb, ob + e);
        if constexpr (NORMS) {
          ee += double(da) * double(da) + double(db) * double(db);
          pp += double(pa) * double(pa) + double(pb) * double(pb);
        }
      });
  if constexpr (NORMS) {
    if (norms) {
      // fixed-order block reduction through the (now free) LDS of the transform
      block_norms<XB>(reinterpret_cast<double*>(lds_mem), ee, pp, norms);
    }
  }
}

template <typename TI, typename T, int N, int BC, bool SUB, int PTM>
__global__ __launch_bounds__(256) void k_xqfwd(const Batch<const TI> in, T* __restrict__ out,
                                                long ostride, long nrows,
                                                const T* __restrict__ tab,
                                                const double* __restrict__ sub,
                                                const int* __restrict__ skip) {
  constexpr int H = N / 2, TPL = FftShape<H, PTM>::TPL, LPB = x_block_threads<N>() / TPL;
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

template <typename T, typename TO, int N, int BC, bool ACCUM, int PTM>
__global__ __launch_bounds__(256) void k_xqinv(const T* __restrict__ in, long istride,
                                                const Batch<TO> out, long nrows,
                                                const T* __restrict__ tab,
                                                const double* __restrict__ sub,
                                                const int* __restrict__ skip,
                                                double* __restrict__ norms) {
  constexpr int XB = x_block_threads<N>();
  constexpr int H = N / 2, TPL = FftShape<H, PTM>::TPL, LPB = XB / TPL;
  constexpr bool NORMS = !std::is_same<T, TO>::value;
  // the norm reduction needs 512 doubles of LDS
  constexpr int LDS_T = 2 * LPB * lds_len<H>();
  constexpr int RED_T = 2 * XB * (int)sizeof(double) / (int)sizeof(T);
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
    if (norms) block_norms<XB>(reinterpret_cast<double*>(lds_mem), ee, pp, norms);
  }
}

// pt: values per thread of the radix schedule, 16 or 8 (a tuning knob; the
// results are the same up to rounding order)
template <int PTM>
static long x_rows_per_block(int n) {
  switch (n) {
#define VP_RPB(NN) \
  case NN: return 2L * (x_block_threads<NN>() / FftShape<NN, PTM>::TPL);
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

#if VP_IN_PART(1)
long xpass_blocks(int nx, int bc, int pt, long nrows) {
  long rpb;
  if (bc == BC_ND || bc == BC_DN) rpb = pt == 8 ? xq_rows<8>(nx) : xq_rows<16>(nx);
  else rpb = pt == 8 ? x_rows_per_block<8>(nx) : x_rows_per_block<16>(nx);
  return rpb > 0 ? (nrows + rpb - 1) / rpb : 0;
}
#endif

template <typename TI, typename T, int BC, bool SUB, int PTM>
static hipError_t launch_xfwd_pt(const Batch<const TI>& in, int nb, T* out, long ostride, int n,
                                 long nrows, const T* tab, const PassOpts& o, hipStream_t st) {
#define VP_XF(NN)                                                                           \
  case NN: {                                                                                \
    const long rpb = 2 * (x_block_threads<NN>() / FftShape<NN, PTM>::TPL);                 \
    hipLaunchKernelGGL((k_xfwd<TI, T, NN, BC, SUB, canon_ptm<NN, PTM>()>),                 \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb),                 \
                       dim3(x_block_threads<NN>()), 0,                                      \
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
    hipLaunchKernelGGL((k_xqfwd<TI, T, NN, BC, SUB, canon_ptm<NN, PTM>()>),                \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb),                 \
                       dim3(x_block_threads<NN>()), 0,                                      \
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
    const long rpb = 2 * (x_block_threads<NN>() / FftShape<NN, PTM>::TPL);                 \
    hipLaunchKernelGGL((k_xinv<T, TO, NN, BC, ACCUM, canon_ptm<NN, PTM>()>),               \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb),                 \
                       dim3(x_block_threads<NN>()), 0,                                      \
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
    hipLaunchKernelGGL((k_xqinv<T, TO, NN, BC, ACCUM, canon_ptm<NN, PTM>()>),              \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb),                 \
                       dim3(x_block_threads<NN>()), 0,                                      \
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

#if VP_IN_PART(1)
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
#endif

#if VP_IN_PART(2)
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
#endif

#if VP_IN_PART(3)
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
#endif

}  // namespace vp
