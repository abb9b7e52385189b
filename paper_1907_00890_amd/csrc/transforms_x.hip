// x passes of the spectral Poisson solve: every x-line (contiguous rows),
// two real lines per complex FFT (real DFT, DCT, sign-alternated DST), or
// one line per half-length FFT (quarter-wave DCT-IV), with the batch,
// shift, accumulation, skip and norm options of the mixed chain.
#include "transform_passes.hpp"

namespace vp {

// Sums over a block's threads of K per-thread values, written to out[0..K):
// a butterfly over the 64 lanes of each wave, then one LDS step over the
// XB / 64 waves (fixed order; red: K * XB / 64 doubles of the block's LDS,
// which the caller no longer needs).
template <int XB, int K>
__device__ __forceinline__ void block_sums(double* red, const double (&v)[K],
                                           double* __restrict__ out) {
  constexpr int NW = XB / 64;
  double w[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    w[i] = v[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) w[i] += __shfl_xor(w[i], o, 64);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) red[i * NW + wid] = w[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < NW; ++j) t += red[i * NW + j];
      out[i] = t;
    }
  }
}

// Partial sums of the mixed chain, kNormSlots doubles per x block of a
// member, at norms + kNormSlots * (member * blocks + block):
//   [0] sum e^2, [1] sum p^2, [2] sum dzf p   (x inverse: e added, p result)
//   [3] sum dzf f (x forward of f) or sum r^2 (x forward in residual mode)
// Element (x, row) of a field lies in z-plane row / ny, of width dzf[row / ny].

// Residual mode of the x forward pass (ResidualArgs): element x of row
// `row` (= y + ny z) is read as r = f - m - L_h p, the defect of the current
// iterate p, in FP64 (L_h of every end type: periodic wrap, wall = no flux,
// outflow = a zero value half a cell beyond the end; z faces at centre
// distances dzc).
// The y and z part of L_h at one row (everything but the x neighbours),
// set up once per row: the neighbour rows' offsets (0 where there is none:
// the difference then reads the row itself, with a zero weight), their
// weights, and the diagonal an outflow end adds (a zero value half a cell
// beyond the end cell).
struct RowStencil {
  long ym, yp, zm, zp;     // element offsets of the neighbour rows
  double wym, wyp, wzm, wzp;
  double dout;             // outflow ends of y and z
};

__device__ __forceinline__ RowStencil row_stencil(const ResidualArgs& a, int nx, int y, int z) {
  RowStencil s;
  const long P = (long)nx * a.ny;
  const bool hym = y > 0 || a.pery, hyp = y + 1 < a.ny || a.pery;
  s.ym = hym ? (y > 0 ? -(long)nx : P - nx) : 0;
  s.yp = hyp ? (y + 1 < a.ny ? (long)nx : nx - P) : 0;
  s.wym = hym ? a.idy2 : 0.0;
  s.wyp = hyp ? a.idy2 : 0.0;
  double d = 0.0;
  if (!hym && (a.outflow & 4)) d += 2.0 * a.idy2;
  if (!hyp && (a.outflow & 8)) d += 2.0 * a.idy2;
  const double ihf = 1.0 / a.dzf[z];
  const bool hzm = z > 0 || a.perz, hzp = z + 1 < a.nz || a.perz;
  s.zm = hzm ? (z > 0 ? -P : (long)(a.nz - 1) * P) : 0;
  s.zp = hzp ? (z + 1 < a.nz ? P : -(long)(a.nz - 1) * P) : 0;
  s.wzm = hzm ? ihf / a.dzc[z > 0 ? z - 1 : a.nz - 1] : 0.0;
  s.wzp = hzp ? ihf / a.dzc[z + 1 < a.nz ? z : a.nz - 1] : 0.0;
  if (!hzm && (a.outflow & 16)) d += 2.0 * ihf * ihf;
  if (!hzp && (a.outflow & 32)) d += 2.0 * ihf * ihf;
  s.dout = d;
  return s;
}

// f - m - L_h p at element x of a row starting at pr (p) with its y and z
// part in rs, every flux as a difference of neighbouring values (the
// rounding of L_h then scales with the differences, not with p); pym / pyp:
// the y-neighbour values where the caller has them (OWN_YM / OWN_YP).
template <int N, bool OWN_YM, bool OWN_YP>
__device__ __forceinline__ double row_residual(const ResidualArgs& a, const double* __restrict__ pr,
                                               const RowStencil& rs, double fc, double m, int x,
                                               double pc, double pym, double pyp) {
  double lx = 0.0;
  if (x + 1 < N) lx += pr[x + 1] - pc;
  else if (a.perx) lx += pr[x + 1 - N] - pc;
  else if (a.outflow & 2) lx -= pc + pc;
  if (x > 0) lx -= pc - pr[x - 1];
  else if (a.perx) lx -= pc - pr[x - 1 + N];
  else if (a.outflow & 1) lx -= pc + pc;
  const double ym = OWN_YM ? pym : pr[x + rs.ym];
  const double yp = OWN_YP ? pyp : pr[x + rs.yp];
  const double lyz = rs.wyp * (yp - pc) - rs.wym * (pc - ym) + rs.wzp * (pr[x + rs.zp] - pc) -
                     rs.wzm * (pc - pr[x + rs.zm]) - rs.dout * pc;
  return fc - m - (a.idx2 * lx + lyz);
}

// ---------------------------------------------------------------------------
// x kernels: a block owns 2*LPB consecutive rows (nrows is even);
// x_block_threads<N>() threads, TPL per line pair
// ---------------------------------------------------------------------------
// T: arithmetic and LDS type; TS: type of the stored spectrum (float in the
// mixed chain, which computes in FP64 and rounds only what it stores).
// RES: residual mode (above; `in` holds f); otherwise the input is read
// unchanged.  With TS != T and `norms` set, slot 3 of the block's partial
// sums receives sum dzf f, or sum r^2 in residual mode.
template <typename TI, typename T, typename TS, int N, int BC, bool RES, int PTM>
__global__ __launch_bounds__(256) void k_xfwd(const Batch<const TI> in, TS* __restrict__ out,
                                               long ostride, long nrows,
                                               const T* __restrict__ tab, const ResidualArgs res,
                                               const int* __restrict__ skip,
                                               double* __restrict__ norms) {
  constexpr int XB = x_block_threads<N>(), TPL = FftShape<N, PTM>::TPL, LPB = XB / TPL;
  constexpr bool SUMS = !std::is_same<T, TS>::value;
  static_assert(2 * LPB * lds_len<N>() * sizeof(T) >= XB * sizeof(double), "LDS for the sums");
  __shared__ T lds_mem[2 * LPB * lds_len<N>()];
  if (skip && skip[blockIdx.y]) return;  // member already converged (whole block)
  const int q = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long ra = (long)blockIdx.x * 2 * LPB + 2 * q;
  const bool ok = ra < nrows;
  const TI* ga = in.p[blockIdx.y] + ra * N;
  const TI* gb = ga + N;
  TS* oa = out + blockIdx.y * ostride + ra * N;
  TS* ob = oa + N;
  double acc = 0.0;
  double m = 0.0, wz = 0.0;
  // residual mode: rows a and b are y and y + 1 of one z-plane (ny even),
  // each the other's y neighbour
  const double* pa = nullptr;
  const double* pb = nullptr;
  RowStencil sa{}, sb{};
  if constexpr (RES) {
    if (res.mean) m = res.mean[blockIdx.y];
    if (ok) {
      pa = res.p.p[blockIdx.y] + ra * N;
      pb = pa + N;
      const int y = (int)(ra % res.ny), z = (int)(ra / res.ny);
      sa = row_stencil(res, N, y, z);
      sb = row_stencil(res, N, y + 1, z);
    }
  }
  if constexpr (SUMS) {
    if (ok && norms) wz = res.dzf[ra / res.ny];  // rows ra, ra + 1 share a plane (ny even)
  }
  XLds<T, N> lds(lds_mem, q, LPB);
  forward_body<T, N, BC, PTM, true>(
      lds, t, tab,
      [&](int e, T& r, T& i) {
        if (!ok) {
          r = T(0);
          i = T(0);
          return;
        }
        if constexpr (RES) {
          const double ca = pa[e], cb = pb[e];
          const double va = row_residual<N, false, true>(res, pa, sa, double(ga[e]), m, e, ca,
                                                         0.0, cb);
          const double vb = row_residual<N, true, false>(res, pb, sb, double(gb[e]), m, e, cb,
                                                         ca, 0.0);
          acc += va * va + vb * vb;
          r = T(va);
          i = T(vb);
        } else {
          r = T(ga[e]);
          i = T(gb[e]);
          if constexpr (SUMS) acc += wz * (double(ga[e]) + double(gb[e]));
        }
      },
      [&](int c0, T a0, T b0, int c1, T a1, T b1) {
        if (!ok) return;
        if constexpr (BC == BC_P) {
          // the packed real DFT pairs positions c0 (even) and c1 = c0 + 1:
          // one vector store per row
          using S2 = typename Vec2<TS>::type;
          S2 va, vb;
          va.x = TS(a0);
          va.y = TS(a1);
          vb.x = TS(b0);
          vb.y = TS(b1);
          *reinterpret_cast<S2*>(oa + c0) = va;
          *reinterpret_cast<S2*>(ob + c0) = vb;
        } else {
          oa[c0] = TS(a0);
          ob[c0] = TS(b0);
          oa[c1] = TS(a1);
          ob[c1] = TS(b1);
        }
      });
  if constexpr (SUMS) {
    if (norms) {
      const double v[1] = {acc};
      block_sums<XB, 1>(reinterpret_cast<double*>(lds_mem), v,
                        norms + kNormSlots * ((long)blockIdx.y * gridDim.x + blockIdx.x) + 3);
    }
  }
}

// With FP32 input (the mixed chain: TS = float, arithmetic in T) and `norms`
// set, each block also writes its sums of e^2, p^2 and dzf p (slots 0-2 of
// its partial sums), where e is the value added (or stored) and p the result.
// ACCUM: out[b] += result - sub[b] (sub may be null); otherwise out = result.
template <typename TS, typename T, typename TO, int N, int BC, bool ACCUM, int PTM>
__global__ __launch_bounds__(256) void k_xinv(const TS* __restrict__ in, long istride,
                                               const Batch<TO> out, long nrows,
                                               const T* __restrict__ tab,
                                               const double* __restrict__ sub,
                                               const int* __restrict__ skip,
                                               double* __restrict__ norms,
                                               const double* __restrict__ dzf, int ny) {
  constexpr int XB = x_block_threads<N>(), TPL = FftShape<N, PTM>::TPL, LPB = XB / TPL;
  constexpr bool NORMS = !std::is_same<TS, TO>::value;
  static_assert(2 * LPB * lds_len<N>() * sizeof(T) >= 3 * XB * sizeof(double), "LDS for the sums");
  __shared__ T lds_mem[2 * LPB * lds_len<N>()];
  if (skip && skip[blockIdx.y]) return;  // member already converged (whole block)
  double ee = 0.0, pp = 0.0, wp = 0.0;
  const int q = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long ra = (long)blockIdx.x * 2 * LPB + 2 * q;
  const bool ok = ra < nrows;
  const TS* ia = in + blockIdx.y * istride + ra * N;
  const TS* ib = ia + N;
  TO* oa = out.p[blockIdx.y] + ra * N;
  TO* ob = oa + N;
  TO shift = TO(0);
  if constexpr (ACCUM) {
    if (sub) shift = TO(sub[blockIdx.y]);
  }
  double wz = 0.0;
  if constexpr (NORMS) {
    if (ok && norms) wz = dzf[ra / ny];  // rows ra, ra + 1 share a plane (ny even)
  }
  XLds<T, N> lds(lds_mem, q, LPB);
  inverse_body<T, N, BC, PTM, true>(
      lds, t, tab,
      [&](int c0, int c1, T& a0, T& b0, T& a1, T& b1) {
        if constexpr (BC == BC_P) {
          // the packed real DFT pairs positions c0 (even) and c1 = c0 + 1:
          // one vector load per row
          using S2 = typename Vec2<TS>::type;
          S2 va{TS(0), TS(0)}, vb{TS(0), TS(0)};
          if (ok) {
            va = *reinterpret_cast<const S2*>(ia + c0);
            vb = *reinterpret_cast<const S2*>(ib + c0);
          }
          a0 = T(va.x);
          a1 = T(va.y);
          b0 = T(vb.x);
          b1 = T(vb.y);
        } else {
          a0 = ok ? T(ia[c0]) : T(0);
          b0 = ok ? T(ib[c0]) : T(0);
          a1 = ok ? T(ia[c1]) : T(0);
          b1 = ok ? T(ib[c1]) : T(0);
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
          wp += wz * (double(pa) + double(pb));
        }
      });
  if constexpr (NORMS) {
    if (norms) {
      const double v[3] = {ee, pp, wp};
      block_sums<XB, 3>(reinterpret_cast<double*>(lds_mem), v,
                        norms + kNormSlots * ((long)blockIdx.y * gridDim.x + blockIdx.x));
    }
  }
}

template <typename TI, typename T, typename TS, int N, int BC, bool RES, int PTM>
__global__ __launch_bounds__(256) void k_xqfwd(const Batch<const TI> in, TS* __restrict__ out,
                                                long ostride, long nrows,
                                                const T* __restrict__ tab, const ResidualArgs res,
                                                const int* __restrict__ skip,
                                                double* __restrict__ norms) {
  constexpr int XB = x_block_threads<N>();
  constexpr int H = N / 2, TPL = FftShape<H, PTM>::TPL, LPB = XB / TPL;
  constexpr bool SUMS = !std::is_same<T, TS>::value;
  constexpr int LDS_T = 2 * LPB * lds_len<H>();
  constexpr int RED_T = XB * (int)sizeof(double) / (int)sizeof(T);
  __shared__ T lds_mem[LDS_T > RED_T ? LDS_T : RED_T];
  if (skip && skip[blockIdx.y]) return;  // member already converged (whole block)
  const int q = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long row = (long)blockIdx.x * LPB + q;
  const bool ok = row < nrows;
  const TI* g = in.p[blockIdx.y] + row * N;
  TS* o = out + blockIdx.y * ostride + row * N;
  double acc = 0.0;
  double m = 0.0, wz = 0.0;
  const double* pr = nullptr;
  RowStencil rs{};
  if constexpr (RES) {
    if (res.mean) m = res.mean[blockIdx.y];
    if (ok) {
      pr = res.p.p[blockIdx.y] + row * N;
      rs = row_stencil(res, N, (int)(row % res.ny), (int)(row / res.ny));
    }
  }
  if constexpr (SUMS) {
    if (ok && norms) wz = res.dzf[row / res.ny];
  }
  XLds<T, H> lds(lds_mem, q, LPB);
  quarter_body<T, N, PTM>(
      lds, t, tab,
      [&](int e, T& v) {
        if (!ok) {
          v = T(0);
          return;
        }
        const int x = qpos<N, BC>(e);
        if constexpr (RES) {
          const double r = row_residual<N, false, false>(res, pr, rs, double(g[x]), m, x, pr[x],
                                                         0.0, 0.0);
          acc += r * r;
          v = T(r);
        } else {
          v = T(g[x]);
          if constexpr (SUMS) acc += wz * double(g[x]);
        }
      },
      [&](int c, T v) {
        if (ok) o[c] = TS(v);
      });
  if constexpr (SUMS) {
    if (norms) {
      const double v[1] = {acc};
      block_sums<XB, 1>(reinterpret_cast<double*>(lds_mem), v,
                        norms + kNormSlots * ((long)blockIdx.y * gridDim.x + blockIdx.x) + 3);
    }
  }
}

template <typename TS, typename T, typename TO, int N, int BC, bool ACCUM, int PTM>
__global__ __launch_bounds__(256) void k_xqinv(const TS* __restrict__ in, long istride,
                                                const Batch<TO> out, long nrows,
                                                const T* __restrict__ tab,
                                                const double* __restrict__ sub,
                                                const int* __restrict__ skip,
                                                double* __restrict__ norms,
                                                const double* __restrict__ dzf, int ny) {
  constexpr int XB = x_block_threads<N>();
  constexpr int H = N / 2, TPL = FftShape<H, PTM>::TPL, LPB = XB / TPL;
  constexpr bool NORMS = !std::is_same<TS, TO>::value;
  // the sums need 3 XB doubles of LDS
  constexpr int LDS_T = 2 * LPB * lds_len<H>();
  constexpr int RED_T = 3 * XB * (int)sizeof(double) / (int)sizeof(T);
  __shared__ T lds_mem[LDS_T > RED_T ? LDS_T : RED_T];
  if (skip && skip[blockIdx.y]) return;  // member already converged (whole block)
  double ee = 0.0, pp = 0.0, wp = 0.0;
  const int q = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long row = (long)blockIdx.x * LPB + q;
  const bool ok = row < nrows;
  const TS* ia = in + blockIdx.y * istride + row * N;
  TO* o = out.p[blockIdx.y] + row * N;
  TO shift = TO(0);
  if constexpr (ACCUM) {
    if (sub) shift = TO(sub[blockIdx.y]);
  }
  double wz = 0.0;
  if constexpr (NORMS) {
    if (ok && norms) wz = dzf[row / ny];
  }
  XLds<T, H> lds(lds_mem, q, LPB);
  quarter_body<T, N, PTM>(
      lds, t, tab, [&](int c, T& v) { v = ok ? T(ia[c]) : T(0); },
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
          wp += wz * double(pv);
        }
      });
  if constexpr (NORMS) {
    if (norms) {
      const double v[3] = {ee, pp, wp};
      block_sums<XB, 3>(reinterpret_cast<double*>(lds_mem), v,
                        norms + kNormSlots * ((long)blockIdx.y * gridDim.x + blockIdx.x));
    }
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

template <typename TI, typename T, typename TS, int BC, bool RES, int PTM>
static hipError_t launch_xfwd_pt(const Batch<const TI>& in, int nb, TS* out, long ostride, int n,
                                 long nrows, const T* tab, const ResidualArgs& ra,
                                 const int* skip, double* norms, hipStream_t st) {
#define VP_XF(NN)                                                                           \
  case NN: {                                                                                \
    const long rpb = 2 * (x_block_threads<NN>() / FftShape<NN, PTM>::TPL);                 \
    hipLaunchKernelGGL((k_xfwd<TI, T, TS, NN, BC, RES, canon_ptm<NN, PTM>()>),             \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb),                 \
                       dim3(x_block_threads<NN>()), 0,                                      \
                       st, in, out, ostride, nrows, tab, ra, skip, norms);                  \
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

template <typename TI, typename T, typename TS, int BC, bool RES, int PTM>
static hipError_t launch_xqfwd_pt(const Batch<const TI>& in, int nb, TS* out, long ostride, int n,
                                  long nrows, const T* tab, const ResidualArgs& ra,
                                  const int* skip, double* norms, hipStream_t st) {
#define VP_XQF(NN)                                                                          \
  case NN: {                                                                                \
    constexpr long rpb = xq_rows_per_block<NN, PTM>();                                      \
    hipLaunchKernelGGL((k_xqfwd<TI, T, TS, NN, BC, RES, canon_ptm<NN, PTM>()>),            \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb),                 \
                       dim3(x_block_threads<NN>()), 0,                                      \
                       st, in, out, ostride, nrows, tab, ra, skip, norms);                  \
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

template <typename TI, typename T, typename TS, int BC, bool RES>
static hipError_t launch_xfwd_bc(const Batch<const TI>& in, int nb, TS* out, long ostride, int n,
                                 long nrows, const T* tab, int pt, const ResidualArgs& ra,
                                 const int* skip, double* norms, hipStream_t st) {
  if constexpr (BC == BC_ND || BC == BC_DN)
    return pt == 8 ? launch_xqfwd_pt<TI, T, TS, BC, RES, 8>(in, nb, out, ostride, n, nrows, tab,
                                                            ra, skip, norms, st)
                   : launch_xqfwd_pt<TI, T, TS, BC, RES, 16>(in, nb, out, ostride, n, nrows, tab,
                                                             ra, skip, norms, st);
  else
    return pt == 8 ? launch_xfwd_pt<TI, T, TS, BC, RES, 8>(in, nb, out, ostride, n, nrows, tab,
                                                           ra, skip, norms, st)
                   : launch_xfwd_pt<TI, T, TS, BC, RES, 16>(in, nb, out, ostride, n, nrows, tab,
                                                            ra, skip, norms, st);
}

template <typename TS, typename T, typename TO, int BC, bool ACCUM, int PTM>
static hipError_t launch_xinv_pt(const TS* in, long istride, const Batch<TO>& out, int nb, int n,
                                 long nrows, const T* tab, const PassOpts& o,
                                 const double* dzf, int ny, hipStream_t st) {
#define VP_XI(NN)                                                                           \
  case NN: {                                                                                \
    const long rpb = 2 * (x_block_threads<NN>() / FftShape<NN, PTM>::TPL);                 \
    hipLaunchKernelGGL((k_xinv<TS, T, TO, NN, BC, ACCUM, canon_ptm<NN, PTM>()>),           \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb),                 \
                       dim3(x_block_threads<NN>()), 0,                                      \
                       st, in, istride, out, nrows, tab, o.sub, o.skip, o.norms, dzf, ny);  \
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

template <typename TS, typename T, typename TO, int BC, bool ACCUM, int PTM>
static hipError_t launch_xqinv_pt(const TS* in, long istride, const Batch<TO>& out, int nb, int n,
                                  long nrows, const T* tab, const PassOpts& o,
                                  const double* dzf, int ny, hipStream_t st) {
#define VP_XQI(NN)                                                                          \
  case NN: {                                                                                \
    constexpr long rpb = xq_rows_per_block<NN, PTM>();                                      \
    hipLaunchKernelGGL((k_xqinv<TS, T, TO, NN, BC, ACCUM, canon_ptm<NN, PTM>()>),          \
                       dim3((unsigned)((nrows + rpb - 1) / rpb), (unsigned)nb),                 \
                       dim3(x_block_threads<NN>()), 0,                                      \
                       st, in, istride, out, nrows, tab, o.sub, o.skip, o.norms, dzf, ny);  \
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

template <typename TS, typename T, typename TO, int BC, bool ACCUM>
static hipError_t launch_xinv_bc(const TS* in, long istride, const Batch<TO>& out, int nb, int n,
                                 long nrows, const T* tab, int pt, const PassOpts& o,
                                 const double* dzf, int ny, hipStream_t st) {
  if constexpr (BC == BC_ND || BC == BC_DN)
    return pt == 8 ? launch_xqinv_pt<TS, T, TO, BC, ACCUM, 8>(in, istride, out, nb, n, nrows, tab,
                                                              o, dzf, ny, st)
                   : launch_xqinv_pt<TS, T, TO, BC, ACCUM, 16>(in, istride, out, nb, n, nrows,
                                                               tab, o, dzf, ny, st);
  else
    return pt == 8 ? launch_xinv_pt<TS, T, TO, BC, ACCUM, 8>(in, istride, out, nb, n, nrows, tab,
                                                             o, dzf, ny, st)
                   : launch_xinv_pt<TS, T, TO, BC, ACCUM, 16>(in, istride, out, nb, n, nrows, tab,
                                                              o, dzf, ny, st);
}

#if VP_IN_PART(1)
hipError_t launch_xfwd_f64(const Batch<const double>& in, int nb, double* out, long ostride,
                           int nx, int bc, long nrows, const double* tab, int pt,
                           hipStream_t st) {
  const ResidualArgs ra{};
  return with_bc(bc, [&](auto B) {
    return launch_xfwd_bc<double, double, double, decltype(B)::value, false>(
        in, nb, out, ostride, nx, nrows, tab, pt, ra, nullptr, nullptr, st);
  });
}

hipError_t launch_xinv_f64(const double* in, long istride, const Batch<double>& out, int nb,
                           int nx, int bc, long nrows, const double* tab, int pt,
                           hipStream_t st) {
  const PassOpts o{};
  return with_bc(bc, [&](auto B) {
    return launch_xinv_bc<double, double, double, decltype(B)::value, false>(
        in, istride, out, nb, nx, nrows, tab, pt, o, nullptr, 1, st);
  });
}
#endif

#if VP_IN_PART(2)
hipError_t launch_xfwd_f32(const Batch<const double>& in, int nb, float* out, long ostride,
                           int nx, int bc, long nrows, const double* tab, int pt,
                           const PassOpts& o, hipStream_t st) {
  if (!o.geo || (o.residual && !o.geo->dzc)) return hipErrorInvalidValue;
  const ResidualArgs& ra = *o.geo;
  return with_bc(bc, [&](auto B) {
    constexpr int BC = decltype(B)::value;
    return o.residual
               ? launch_xfwd_bc<double, double, float, BC, true>(in, nb, out, ostride, nx, nrows,
                                                                 tab, pt, ra, o.skip, o.norms, st)
               : launch_xfwd_bc<double, double, float, BC, false>(in, nb, out, ostride, nx, nrows,
                                                                  tab, pt, ra, o.skip, o.norms, st);
  });
}
#endif

#if VP_IN_PART(3)
hipError_t launch_xinv_f32(const float* in, long istride, const Batch<double>& out, int nb,
                           int nx, int bc, long nrows, bool accum, const double* tab, int pt,
                           const PassOpts& o, hipStream_t st) {
  if (!o.geo) return hipErrorInvalidValue;
  const double* dzf = o.geo->dzf;
  const int ny = o.geo->ny;
  return with_bc(bc, [&](auto B) {
    constexpr int BC = decltype(B)::value;
    return accum ? launch_xinv_bc<float, double, double, BC, true>(in, istride, out, nb, nx, nrows,
                                                                   tab, pt, o, dzf, ny, st)
                 : launch_xinv_bc<float, double, double, BC, false>(in, istride, out, nb, nx,
                                                                    nrows, tab, pt, o, dzf, ny, st);
  });
}
#endif

}  // namespace vp
