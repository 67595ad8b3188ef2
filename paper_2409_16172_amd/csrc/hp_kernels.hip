// HIP kernels for gfx950: the interpolated preconditioner Q_M (Eqn. 403/405),
// the finite-difference operator P_N (Section 5) and the FP64 Krylov kernels of
// restarted GMRES.
//
// Preconditioner apply, d = 2 (grid n0 x n1, axis 1 contiguous):
//   pass A  forward FFT of every row                       v  -> t
//   pass B  per tile of columns: forward FFT along axis 0, then for each of the
//           K nodes the symbol multiply (computed on the fly from two 1-D tables
//           of lambda) and the inverse FFT along axis 0     t  -> K node fields
//   pass C  per row: inverse FFT of the K node rows and the combine with the two
//           non-zero piecewise-linear weights of each point  K fields -> u
// d = 3 adds the forward and inverse transforms along the middle axis as plain
// strided passes (A' and M) between A/B and B/C.
#include "hp_internal.h"

namespace hp {

template <typename R, typename S>
__device__ __forceinline__ cpx<R> cvt(cpx<S> a) {
  return {(R)a.re, (R)a.im};
}

// Rows (contiguous axis): G lines of length N per workgroup of 256 threads
// (one line per workgroup when a line needs 256 threads or more).
#ifndef HP_ROWC_THREADS
#define HP_ROWC_THREADS 128
#endif
#ifndef HP_PREFETCH_C
#define HP_PREFETCH_C 0
#endif
template <typename R, int N, int WG = 256>
struct RowCfg {
  static constexpr int E = elems_per_thread<R>(N);
  static constexpr int T = N / E;
  static constexpr int G = T >= WG ? 1 : WG / T;
  static constexpr int THREADS = G * T;
  static constexpr int LDS = (N > E) ? G * lds_elems<R>(N) : 1;
};
template <typename R, int N>
using CombCfg = RowCfg<R, N, HP_ROWC_THREADS>;

// Column tiles (strided axis): TC adjacent columns per workgroup.  Plain
// passes aim at 64-byte row segments; the symbol pass, whose workgroups stay
// resident through K transforms, uses the smallest workgroup (>= 256 threads)
// that still reads and writes 32-byte row segments, so that more independent
// workgroups share a CU.
template <typename R, int N, int MAXT, int SEG = 64>
struct ColCfg {
  static constexpr int E = elems_per_thread<R>(N);
  static constexpr int T = N / E;
  static constexpr int TC0 = SEG / (2 * (int)sizeof(R));
  static constexpr int THR0 = TC0 * T < 256 ? 256 : TC0 * T;
  static constexpr int THREADS = THR0 > MAXT ? MAXT : THR0;
  static constexpr int TC = THREADS / T;
  static constexpr int LDS = (N > E) ? TC * lds_elems<R>(N) : 1;
};
#ifndef HP_SYM_MAXT
#define HP_SYM_MAXT 512
#endif
#ifndef HP_SYM_SEG
#define HP_SYM_SEG 32
#endif
#ifndef HP_XCD_REMAP
#define HP_XCD_REMAP 1
#endif
template <int MODE>
constexpr int cols_max_threads() { return MODE == 1 ? HP_SYM_MAXT : 1024; }

// ---------------------------------------------------------------- pass A
template <typename R, typename TI, int N>
__global__ __launch_bounds__((RowCfg<R, N>::THREADS)) void k_rows_fwd(const cpx<TI>* __restrict__ in,
                                                                  cpx<R>* __restrict__ out, int rows,
                                                                  size_t in_rs, size_t out_rs,
                                                                  const cpx<R>* __restrict__ tw,
                                                                  const int* __restrict__ skip) {
  using C = RowCfg<R, N>;
  __shared__ cpx<R> lds[C::LDS];
  const int rhs = blockIdx.y;
  if (skip != nullptr && skip[rhs] != 0) return;
  const int g = threadIdx.x / C::T, j = threadIdx.x % C::T;
  const int row = blockIdx.x * C::G + g;
  const bool act = row < rows;
  const cpx<TI>* src = in + (size_t)rhs * in_rs + (size_t)row * N;
  cpx<R> x[C::E];
#pragma unroll
  for (int s = 0; s < C::E; ++s) x[s] = act ? cvt<R>(src[j + C::T * s]) : cpx<R>{0, 0};
  fft<R, N, -1, true>(x, lds + g * lds_elems<R>(N), j, tw);
  if (act) {
    cpx<R>* dst = out + (size_t)rhs * out_rs + (size_t)row * N;
#pragma unroll
    for (int s = 0; s < C::E; ++s) dst[j + C::T * s] = x[s];
  }
}

// ---------------------------------------------------------------- strided passes
// 1/x for finite x > 0: hardware reciprocal estimate refined by Newton-Raphson
// steps r <- r + r (1 - x r) (two in FP64, one in FP32).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  const float e = __builtin_fmaf(-x, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}

// Symbol multiply of one node on the elements a thread holds.  The denominator
// A_n - g_n lambda is formed in FP64 (it cancels near |xi| = omega/|gamma_n|),
// then reciprocated in the working precision.
template <typename R, int E>
__device__ __forceinline__ void symbol_mul(const cpx<R> (&vh)[E], cpx<R> (&x)[E], const double (&lam)[E],
                                           NodeConst nc, double scale) {
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const double dre = nc.are - nc.gre * lam[s];
    const double dim = nc.aim - nc.gim * lam[s];
    cpx<R> q;
    if constexpr (sizeof(R) == 8) {
      const double inv = scale * recip(dre * dre + dim * dim);
      q = {dre * inv, -dim * inv};
    } else {
      const float fr = (float)dre, fi = (float)dim;
      const float inv = (float)scale * recip(fr * fr + fi * fi);
      q = {fr * inv, -fi * inv};
    }
    x[s] = cmul(vh[s], q);
  }
}

template <typename R, typename TI, int N, int DIR, int MODE>
__global__ __launch_bounds__((ColCfg<R, N, cols_max_threads<MODE>(), MODE == 1 ? HP_SYM_SEG : 64>::THREADS)) void k_cols(
    const cpx<TI>* __restrict__ in, cpx<R>* __restrict__ out, int S, int nfields, size_t in_rs,
    size_t out_rs, size_t in_fs, size_t out_fs, const cpx<R>* __restrict__ tw,
    const int* __restrict__ skip, const double* __restrict__ lam_ax, const double* __restrict__ lam_in,
    const NodeConst* __restrict__ nodes, int K, double scale, const uint16_t* __restrict__ store_mask,
    const uint8_t* __restrict__ slab_need) {
  using C = ColCfg<R, N, cols_max_threads<MODE>(), MODE == 1 ? HP_SYM_SEG : 64>;
  __shared__ cpx<R> lds[C::LDS];
  const int z = blockIdx.z;
  const int rhs = (MODE == 0) ? z / nfields : z;
  const int fld = (MODE == 0) ? z % nfields : 0;
  if (skip != nullptr && skip[rhs] != 0) return;
  // plain passes over node fields: slabs whose points never use this node are skipped
  if (MODE == 0 && slab_need != nullptr && slab_need[(size_t)fld * gridDim.y + blockIdx.y] == 0) return;
  const int g = threadIdx.x % C::TC, j = threadIdx.x / C::TC;
  // Workgroups are dispatched round-robin over the 8 XCDs (each with its own
  // L2).  Give the workgroups of one XCD consecutive column tiles so that tiles
  // sharing cache lines meet in the same L2.
  int tile = blockIdx.x;
#if HP_XCD_REMAP
  if ((gridDim.x & 7) == 0) tile = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
#endif
  const int c = tile * C::TC + g;
  const bool act = c < S;
  const size_t obase = (size_t)blockIdx.y * N * S + c;
  const cpx<TI>* src = in + (size_t)rhs * in_rs + (size_t)fld * in_fs + obase;
  cpx<R>* lg = lds + g;   // the TC columns are interleaved in LDS
  cpx<R> x[C::E];
#pragma unroll
  for (int s = 0; s < C::E; ++s)
    x[s] = act ? cvt<R>(src[(size_t)(j + C::T * s) * S]) : cpx<R>{0, 0};
  if constexpr (MODE == 0) {
    fft<R, N, DIR, false, C::TC>(x, lg, j, tw);
    if (act) {
      cpx<R>* dst = out + (size_t)rhs * out_rs + (size_t)fld * out_fs + obase;
#pragma unroll
      for (int s = 0; s < C::E; ++s) dst[(size_t)(j + C::T * s) * S] = x[s];
    }
  } else {
    fft<R, N, -1, false, C::TC>(x, lg, j, tw);
    cpx<R> vh[C::E];
    double lam[C::E];
    const double lc = act ? lam_in[c] : 0.0;
#pragma unroll
    for (int s = 0; s < C::E; ++s) {
      vh[s] = x[s];
      lam[s] = lam_ax[j + C::T * s] + lc;
    }
    cpx<R>* dst = out + (size_t)rhs * out_rs + obase;
    for (int n = 0; n < K; ++n) {
      symbol_mul<R, C::E>(vh, x, lam, nodes[n], scale);
      fft<R, N, +1, false, C::TC>(x, lg, j, tw);
      // bit s: some point of axis-0 index j + T*s uses node n (else the row is never read)
      const uint32_t m = act ? (uint32_t)store_mask[n * C::T + j] : 0u;
#pragma unroll
      for (int s = 0; s < C::E; ++s)
        if ((m >> s) & 1u) dst[(size_t)n * out_fs + (size_t)(j + C::T * s) * S] = x[s];
    }
  }
}

// ---------------------------------------------------------------- pass C
// Interpolation record of one point: pos >= 0 encodes the real-axis segment
// seg + t (weights 1-t on node seg, t on node seg+1); pos < 0 encodes the layer
// segment, -(1 + j + t): weights 1-t on the lower layer node (c_o itself for
// j = 0) and t on layer node j+1 (Eqn. 405 with Re gamma = c_o in the layer).
__device__ __forceinline__ void decode_pos(double p, int M, int Mt, int mo, int& A, int& B, double& t) {
  if (p >= 0.0) {
    if (M == 1) {
      A = 0; B = 0; t = 0.0;
      return;
    }
    int s = (int)p;
    if (s > M - 2) s = M - 2;
    A = s; B = s + 1; t = p - (double)s;
  } else {
    const double q = -p - 1.0;
    int s = (int)q;
    if (s > Mt - 1) s = Mt - 1;
    A = (s == 0) ? mo : M + s - 1; B = M + s; t = q - (double)s;
  }
}

template <typename R, typename TO, int N, bool ACC>
__global__ __launch_bounds__((CombCfg<R, N>::THREADS)) void k_rows_combine(
    const cpx<R>* __restrict__ fields, size_t fs, size_t frs, const double* __restrict__ pos,
    const uint64_t* __restrict__ grpmask, const uint64_t* __restrict__ rowmask, cpx<TO>* __restrict__ out,
    size_t out_rs, int rows, int K, int M, int Mt, int mo, const cpx<R>* __restrict__ tw,
    const int* __restrict__ skip) {
  using C = CombCfg<R, N>;
  __shared__ cpx<R> lds[C::LDS];
  const int rhs = blockIdx.y;
  if (skip != nullptr && skip[rhs] != 0) return;
  const int g = threadIdx.x / C::T, j = threadIdx.x % C::T;
  const int row = blockIdx.x * C::G + g;
  const bool act = row < rows;
  const size_t rbase = (size_t)row * N;
  int ab[C::E];
  R tt[C::E];
  cpx<R> acc[C::E];
#pragma unroll
  for (int s = 0; s < C::E; ++s) {
    int A = -1, B = -1;
    double t = 0.0;
    if (act) decode_pos(pos[rbase + j + C::T * s], M, Mt, mo, A, B, t);
    ab[s] = (A & 0xff) | ((B & 0xff) << 8);
    tt[s] = (R)t;
    acc[s] = {0, 0};
  }
  const uint64_t mask = grpmask[blockIdx.x];
  const uint64_t rmask = act ? rowmask[row] : 0ull;
  const cpx<R>* fr = fields + (size_t)rhs * frs + rbase;
  cpx<R>* lg = lds + g * lds_elems<R>(N);
  // Nodes no point of this group uses are skipped; rows that do not use a node
  // read zeros (pass B did not write them).  The next used node's row is loaded
  // while the current one is transformed.
  auto next_node = [&](int n) {
    while (n < K && ((mask >> n) & 1ull) == 0) ++n;
    return n;
  };
  cpx<R> nx[C::E];
  int n = next_node(0);
  if (!HP_PREFETCH_C && n < K) {
    // loaded at the top of the loop instead
  } else if (n < K) {
    const bool ld = ((rmask >> n) & 1ull) != 0;
#pragma unroll
    for (int s = 0; s < C::E; ++s) nx[s] = ld ? fr[(size_t)n * fs + j + C::T * s] : cpx<R>{0, 0};
  }
  for (; n < K;) {
    cpx<R> x[C::E];
    const int n2 = next_node(n + 1);
    if (!HP_PREFETCH_C) {
      const bool ld = ((rmask >> n) & 1ull) != 0;
#pragma unroll
      for (int s = 0; s < C::E; ++s) x[s] = ld ? fr[(size_t)n * fs + j + C::T * s] : cpx<R>{0, 0};
    } else {
#pragma unroll
      for (int s = 0; s < C::E; ++s) x[s] = nx[s];
    }
    if (HP_PREFETCH_C && n2 < K) {
      const bool ld = ((rmask >> n2) & 1ull) != 0;
#pragma unroll
      for (int s = 0; s < C::E; ++s) nx[s] = ld ? fr[(size_t)n2 * fs + j + C::T * s] : cpx<R>{0, 0};
    }
    fft<R, N, +1, true>(x, lg, j, tw);
#pragma unroll
    for (int s = 0; s < C::E; ++s) {
      const int A = ab[s] & 0xff, B = (ab[s] >> 8) & 0xff;
      const R w = (A == n ? (R)1 - tt[s] : (R)0) + (B == n ? tt[s] : (R)0);
      acc[s].re += w * x[s].re;
      acc[s].im += w * x[s].im;
    }
    n = n2;
  }
  if (act) {
    cpx<TO>* dst = out + (size_t)rhs * out_rs + rbase;
#pragma unroll
    for (int s = 0; s < C::E; ++s) {
      if constexpr (ACC) {
        cpx<TO> o = dst[j + C::T * s];
        dst[j + C::T * s] = {o.re + (TO)acc[s].re, o.im + (TO)acc[s].im};
      } else {
        dst[j + C::T * s] = cvt<TO>(acc[s]);
      }
    }
  }
}

// ---------------------------------------------------------------- dispatch
template <template <int> class F, typename... Args>
hipError_t dispatch_n(int n, Args... args) {
  switch (n) {
    case 8: return F<8>::run(args...);
    case 16: return F<16>::run(args...);
    case 32: return F<32>::run(args...);
    case 64: return F<64>::run(args...);
    case 128: return F<128>::run(args...);
    case 256: return F<256>::run(args...);
    case 512: return F<512>::run(args...);
    case 1024: return F<1024>::run(args...);
    case 2048: return F<2048>::run(args...);
    case 4096: return F<4096>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

template <typename R, typename TI>
struct RowsFwdL {
  template <int N>
  struct F {
    static hipError_t run(const void* in, void* out, int rows, size_t in_rs, size_t out_rs, int nrhs,
                          const void* tw, const int* skip, hipStream_t st) {
      using C = RowCfg<R, N>;
      dim3 grid((rows + C::G - 1) / C::G, nrhs);
      hipLaunchKernelGGL((k_rows_fwd<R, TI, N>), grid, dim3(C::THREADS), 0, st, (const cpx<TI>*)in,
                         (cpx<R>*)out, rows, in_rs, out_rs, (const cpx<R>*)tw, skip);
      return hipGetLastError();
    }
  };
};

hipError_t launch_rows_fwd(int real_kind, int in_kind, int n, const void* in, void* out, int rows,
                           size_t in_rs, size_t out_rs, int nrhs, const void* tw, const int* skip,
                           hipStream_t st) {
  if (real_kind == 0) {
    if (in_kind != 0) return hipErrorInvalidValue;
    return dispatch_n<RowsFwdL<double, double>::F>(n, in, out, rows, in_rs, out_rs, nrhs, tw, skip, st);
  }
  if (in_kind == 0)
    return dispatch_n<RowsFwdL<float, double>::F>(n, in, out, rows, in_rs, out_rs, nrhs, tw, skip, st);
  return dispatch_n<RowsFwdL<float, float>::F>(n, in, out, rows, in_rs, out_rs, nrhs, tw, skip, st);
}

template <typename R>
struct ColsL {
  template <int N>
  struct F {
    static hipError_t run(const ColsArgs& a, hipStream_t st) {
      using C0 = ColCfg<R, N, cols_max_threads<0>()>;
      using C1 = ColCfg<R, N, cols_max_threads<1>(), HP_SYM_SEG>;
      if constexpr (sizeof(R) == 8 && N > 2048) {
        return hipErrorInvalidValue;   // the FP64 column tile would not fit in LDS
      } else {
        const int TC = a.mode == 1 ? C1::TC : C0::TC;
        dim3 grid((a.S + TC - 1) / TC, a.outer, a.mode == 0 ? a.nrhs * a.nfields : a.nrhs);
        const cpx<R>* in = (const cpx<R>*)a.in;
        cpx<R>* out = (cpx<R>*)a.out;
        const cpx<R>* tw = (const cpx<R>*)a.tw;
        if (a.mode == 1)
          hipLaunchKernelGGL((k_cols<R, R, N, -1, 1>), grid, dim3(C1::THREADS), 0, st, in, out, a.S,
                             a.nfields, a.in_rs, a.out_rs, a.in_fs, a.out_fs, tw, a.skip, a.lam_ax,
                             a.lam_in, a.nodes, a.K, a.scale, a.store_mask, a.slab_need);
        else if (a.dir < 0)
          hipLaunchKernelGGL((k_cols<R, R, N, -1, 0>), grid, dim3(C0::THREADS), 0, st, in, out, a.S,
                             a.nfields, a.in_rs, a.out_rs, a.in_fs, a.out_fs, tw, a.skip, a.lam_ax,
                             a.lam_in, a.nodes, a.K, a.scale, a.store_mask, a.slab_need);
        else
          hipLaunchKernelGGL((k_cols<R, R, N, +1, 0>), grid, dim3(C0::THREADS), 0, st, in, out, a.S,
                             a.nfields, a.in_rs, a.out_rs, a.in_fs, a.out_fs, tw, a.skip, a.lam_ax,
                             a.lam_in, a.nodes, a.K, a.scale, a.store_mask, a.slab_need);
        return hipGetLastError();
      }
    }
  };
};

hipError_t launch_cols(const ColsArgs& a, hipStream_t st) {
  if (a.real_kind == 0) return dispatch_n<ColsL<double>::F>(a.n, a, st);
  return dispatch_n<ColsL<float>::F>(a.n, a, st);
}

template <typename R, typename TO, bool ACC>
struct CombineL {
  template <int N>
  struct F {
    static hipError_t run(const CombineArgs& a, hipStream_t st) {
      using C = CombCfg<R, N>;
      dim3 grid((a.rows + C::G - 1) / C::G, a.nrhs);
      hipLaunchKernelGGL((k_rows_combine<R, TO, N, ACC>), grid, dim3(C::THREADS), 0, st,
                         (const cpx<R>*)a.fields, a.fs, a.frs, a.pos, a.grpmask, a.rowmask, (cpx<TO>*)a.out,
                         a.out_rs, a.rows, a.K, a.M, a.Mt, a.mo, (const cpx<R>*)a.tw, a.skip);
      return hipGetLastError();
    }
  };
};

hipError_t launch_combine(const CombineArgs& a, hipStream_t st) {
  if (a.real_kind == 0) {
    if (a.out_kind != 0) return hipErrorInvalidValue;
    if (a.accumulate) return dispatch_n<CombineL<double, double, true>::F>(a.n, a, st);
    return dispatch_n<CombineL<double, double, false>::F>(a.n, a, st);
  }
  if (a.out_kind == 0) {
    if (a.accumulate) return dispatch_n<CombineL<float, double, true>::F>(a.n, a, st);
    return dispatch_n<CombineL<float, double, false>::F>(a.n, a, st);
  }
  if (a.accumulate) return hipErrorInvalidValue;
  return dispatch_n<CombineL<float, float, false>::F>(a.n, a, st);
}

template <typename R>
int group_rows(int n) {
  switch (n) {
    case 8: return CombCfg<R, 8>::G;
    case 16: return CombCfg<R, 16>::G;
    case 32: return CombCfg<R, 32>::G;
    case 64: return CombCfg<R, 64>::G;
    case 128: return CombCfg<R, 128>::G;
    case 256: return CombCfg<R, 256>::G;
    case 512: return CombCfg<R, 512>::G;
    case 1024: return CombCfg<R, 1024>::G;
    case 2048: return CombCfg<R, 2048>::G;
    case 4096: return CombCfg<R, 4096>::G;
    default: return 1;
  }
}

template <typename R>
int sym_line_threads(int n) {
  switch (n) {
    case 8: return ColCfg<R, 8, cols_max_threads<1>(), HP_SYM_SEG>::T;
    case 16: return ColCfg<R, 16, cols_max_threads<1>(), HP_SYM_SEG>::T;
    case 32: return ColCfg<R, 32, cols_max_threads<1>(), HP_SYM_SEG>::T;
    case 64: return ColCfg<R, 64, cols_max_threads<1>(), HP_SYM_SEG>::T;
    case 128: return ColCfg<R, 128, cols_max_threads<1>(), HP_SYM_SEG>::T;
    case 256: return ColCfg<R, 256, cols_max_threads<1>(), HP_SYM_SEG>::T;
    case 512: return ColCfg<R, 512, cols_max_threads<1>(), HP_SYM_SEG>::T;
    case 1024: return ColCfg<R, 1024, cols_max_threads<1>(), HP_SYM_SEG>::T;
    case 2048: return ColCfg<R, 2048, cols_max_threads<1>(), HP_SYM_SEG>::T;
    case 4096: return ColCfg<R, 4096, cols_max_threads<1>(), HP_SYM_SEG>::T;
    default: return 1;
  }
}

int symbol_pass_line_threads(int real_kind, int n) {
  return real_kind == 0 ? sym_line_threads<double>(n) : sym_line_threads<float>(n);
}

int combine_group_rows(int real_kind, int n) {
  return real_kind == 0 ? group_rows<double>(n) : group_rows<float>(n);
}

// ---------------------------------------------------------------- stencil
// (P u)(x) = gamma^2 sum_j (u(x+e_j) + u(x-e_j)) / h_j^2 + beta u(x),
// beta = omega^2 + i omega a - 2 gamma^2 sum_j 1/h_j^2; periodic indices.
// coef holds {gamma^2, beta} per point.
template <typename R, typename TI, typename TO, int DIM, bool RESID>
__global__ __launch_bounds__(256) void k_stencil(const cpx<TI>* __restrict__ u, cpx<TO>* __restrict__ y,
                                                 const cpx<R>* __restrict__ coef,
                                                 const cpx<double>* __restrict__ f, int n0, int n1,
                                                 int n2, R ih0, R ih1, R ih2, size_t u_rs, size_t y_rs,
                                                 const int* __restrict__ skip) {
  const int rhs = blockIdx.y;
  if (skip != nullptr && skip[rhs] != 0) return;
  const size_t npts = (size_t)n0 * n1 * (DIM == 3 ? n2 : 1);
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= npts) return;
  const cpx<TI>* ur = u + (size_t)rhs * u_rs;
  cpx<R> lap;
  if constexpr (DIM == 2) {
    const int i1 = (int)(i % n1), i0 = (int)(i / n1);
    const size_t r0 = (size_t)i0 * n1;
    const size_t up = (size_t)((i0 + 1) & (n0 - 1)) * n1, dn = (size_t)((i0 - 1) & (n0 - 1)) * n1;
    const cpx<R> a = cvt<R>(ur[r0 + ((i1 + 1) & (n1 - 1))]), b = cvt<R>(ur[r0 + ((i1 - 1) & (n1 - 1))]);
    const cpx<R> c = cvt<R>(ur[up + i1]), d = cvt<R>(ur[dn + i1]);
    lap = {(a.re + b.re) * ih1 + (c.re + d.re) * ih0, (a.im + b.im) * ih1 + (c.im + d.im) * ih0};
  } else {
    const int i2 = (int)(i % n2);
    const int i1 = (int)((i / n2) % n1);
    const int i0 = (int)(i / ((size_t)n1 * n2));
    const size_t s1 = n2, s0 = (size_t)n1 * n2;
    const size_t b0 = (size_t)i0 * s0, b1 = (size_t)i1 * s1;
    const cpx<R> a = cvt<R>(ur[b0 + b1 + ((i2 + 1) & (n2 - 1))]), b = cvt<R>(ur[b0 + b1 + ((i2 - 1) & (n2 - 1))]);
    const cpx<R> c = cvt<R>(ur[b0 + (size_t)((i1 + 1) & (n1 - 1)) * s1 + i2]);
    const cpx<R> d = cvt<R>(ur[b0 + (size_t)((i1 - 1) & (n1 - 1)) * s1 + i2]);
    const cpx<R> e = cvt<R>(ur[(size_t)((i0 + 1) & (n0 - 1)) * s0 + b1 + i2]);
    const cpx<R> q = cvt<R>(ur[(size_t)((i0 - 1) & (n0 - 1)) * s0 + b1 + i2]);
    lap = {(a.re + b.re) * ih2 + (c.re + d.re) * ih1 + (e.re + q.re) * ih0,
           (a.im + b.im) * ih2 + (c.im + d.im) * ih1 + (e.im + q.im) * ih0};
  }
  const cpx<R> g2 = coef[2 * i], be = coef[2 * i + 1];
  const cpx<R> uc = cvt<R>(ur[i]);
  cpx<R> r = cadd(cmul(g2, lap), cmul(be, uc));
  if constexpr (RESID) {
    const cpx<double> fv = f[(size_t)rhs * u_rs + i];
    y[(size_t)rhs * y_rs + i] = {(TO)(fv.re - (double)r.re), (TO)(fv.im - (double)r.im)};
  } else {
    y[(size_t)rhs * y_rs + i] = cvt<TO>(r);
  }
}

hipError_t launch_stencil(const StencilArgs& a, hipStream_t st) {
  const size_t npts = (size_t)a.n[0] * a.n[1] * (a.dim == 3 ? a.n[2] : 1);
  dim3 grid((unsigned)((npts + 255) / 256), a.nrhs);
  const int n2 = a.dim == 3 ? a.n[2] : 1;
#define HP_STENCIL(R, TI, TO, D, RES)                                                                    \
  hipLaunchKernelGGL((k_stencil<R, TI, TO, D, RES>), grid, dim3(256), 0, st, (const cpx<TI>*)a.u,         \
                     (cpx<TO>*)a.y, (const cpx<R>*)a.coef, (const cpx<double>*)a.f, a.n[0], a.n[1], n2,  \
                     (R)a.ih2[0], (R)a.ih2[1], (R)a.ih2[2], a.u_rs, a.y_rs, a.skip)
  if (a.dim == 2) {
    switch (a.kind) {
      case 0: HP_STENCIL(double, double, double, 2, false); break;
      case 1: HP_STENCIL(float, float, float, 2, false); break;
      case 2: HP_STENCIL(float, float, double, 2, false); break;
      case 3: HP_STENCIL(double, double, double, 2, true); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (a.kind) {
      case 0: HP_STENCIL(double, double, double, 3, false); break;
      case 1: HP_STENCIL(float, float, float, 3, false); break;
      case 2: HP_STENCIL(float, float, double, 3, false); break;
      case 3: HP_STENCIL(double, double, double, 3, true); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef HP_STENCIL
  return hipGetLastError();
}

// ---------------------------------------------------------------- Krylov kernels
// All sums are deterministic: each block reduces its own fixed range of points
// in a fixed order (wavefront butterfly, then waves in order) and the partial
// sums of the kRedBlocks blocks of a right-hand side are added in a fixed order.
constexpr int kChunk = 16;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Reduce `cnt` complex values per thread over the block and write them to part.
template <int CNT>
__device__ __forceinline__ void block_reduce_write(cpx<double> (&acc)[CNT], int cnt, cpx<double>* dst) {
  __shared__ double red[kRedThreads / 64][2 * CNT];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < CNT; ++v) {
    if (v < cnt) {
      const double re = wave_sum(acc[v].re), im = wave_sum(acc[v].im);
      if (lane == 0) { red[wv][2 * v] = re; red[wv][2 * v + 1] = im; }
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int w = 0; w < kRedThreads / 64; ++w) { re += red[w][2 * threadIdx.x]; im += red[w][2 * threadIdx.x + 1]; }
    dst[threadIdx.x] = {re, im};
  }
  __syncthreads();
}

// part[rhs][blk][0..nvec-1] = V_v^H w (partial), part[..][nvec] = ||w||^2 (partial).
__global__ __launch_bounds__(kRedThreads) void k_dots(const cpx<double>* __restrict__ V, size_t npts,
                                                       size_t vrs, const cpx<double>* __restrict__ w,
                                                       size_t wrs, int nvec, cpx<double>* __restrict__ part,
                                                       const int* __restrict__ skip) {
  const int rhs = blockIdx.y;
  if (skip != nullptr && skip[rhs] != 0) return;
  const cpx<double>* Vr = V + (size_t)rhs * vrs;
  const cpx<double>* wr = w + (size_t)rhs * wrs;
  cpx<double>* pr = part + ((size_t)rhs * kRedBlocks + blockIdx.x) * kPartSlots;
  const size_t stride = (size_t)kRedBlocks * kRedThreads;
  {
    cpx<double> nrm[1] = {{0.0, 0.0}};
    for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < npts; i += stride) {
      const cpx<double> a = wr[i];
      nrm[0].re += a.re * a.re + a.im * a.im;
    }
    block_reduce_write<1>(nrm, 1, pr + nvec);
  }
  for (int c0 = 0; c0 < nvec; c0 += kChunk) {
    const int cnt = nvec - c0 < kChunk ? nvec - c0 : kChunk;
    cpx<double> acc[kChunk];
#pragma unroll
    for (int v = 0; v < kChunk; ++v) acc[v] = {0.0, 0.0};
    for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < npts; i += stride) {
      const cpx<double> a = wr[i];
#pragma unroll
      for (int v = 0; v < kChunk; ++v) {
        if (v < cnt) {
          const cpx<double> b = Vr[(size_t)(c0 + v) * npts + i];
          acc[v].re += b.re * a.re + b.im * a.im;     // conj(b) * a
          acc[v].im += b.re * a.im - b.im * a.re;
        }
      }
    }
    block_reduce_write<kChunk>(acc, cnt, pr + c0);
  }
}

// Sum the block partials of `cnt` slots of right-hand side `rhs` into sums[]
// (one 1024-thread block; wave w handles slots w, w+16, ...).
__device__ void reduce_slots(const cpx<double>* __restrict__ part, int rhs, int cnt, cpx<double>* sums) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const cpx<double>* pr = part + (size_t)rhs * kRedBlocks * kPartSlots;
  for (int s = wv; s < cnt; s += nw) {
    double re = 0.0, im = 0.0;
    for (int b = lane; b < kRedBlocks; b += 64) {
      re += pr[(size_t)b * kPartSlots + s].re;
      im += pr[(size_t)b * kPartSlots + s].im;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) sums[s] = {re, im};
  }
  __syncthreads();
}

__device__ __forceinline__ double cabs2(cpx<double> a) { return a.re * a.re + a.im * a.im; }

// ||f|| once per solve; target = rtol ||f||.
__global__ __launch_bounds__(1024) void k_fnorm(const cpx<double>* part, KState* state, int* done,
                                                double rtol) {
  __shared__ cpx<double> sums[1];
  const int rhs = blockIdx.x;
  reduce_slots(part, rhs, 1, sums);
  if (threadIdx.x == 0) {
    KState& S = state[rhs];
    S.fnorm = sqrt(sums[0].re);
    S.target = rtol * S.fnorm;
    S.iters = 0;
    S.cycles = 0;
    S.relres = S.fnorm > 0.0 ? 1.0 : 0.0;
    done[rhs] = S.fnorm > 0.0 ? 0 : 1;
  }
}

// Cycle start: beta = ||r||, convergence test on the true residual.
__global__ __launch_bounds__(1024) void k_cycle_start(const cpx<double>* part, KState* state, int* done,
                                                      int* skip_step, double rtol) {
  __shared__ cpx<double> sums[1];
  const int rhs = blockIdx.x;
  if (done[rhs]) {
    if (threadIdx.x == 0) skip_step[rhs] = 1;
    return;
  }
  reduce_slots(part, rhs, 1, sums);
  if (threadIdx.x == 0) {
    KState& S = state[rhs];
    const double beta = sqrt(sums[0].re);
    S.beta = beta;
    S.relres = S.fnorm > 0.0 ? beta / S.fnorm : 0.0;
    if (S.relres <= rtol || beta == 0.0) {
      done[rhs] = 1;
      skip_step[rhs] = 1;
    } else {
      S.cycles += 1;
      S.k = 0;
      S.reorth = 0;
      for (int i = 0; i <= kMaxRestart; ++i) S.g[i] = {0.0, 0.0};
      S.g[0] = {beta, 0.0};
      skip_step[rhs] = 0;
    }
  }
}

__global__ __launch_bounds__(256) void k_scale_v0(cpx<double>* V, size_t npts, size_t vrs, const KState* state,
                                                  const int* done) {
  const int rhs = blockIdx.y;
  if (done[rhs]) return;
  const double s = 1.0 / state[rhs].beta;
  cpx<double>* v = V + (size_t)rhs * vrs;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < npts; i += (size_t)gridDim.x * 256)
    v[i] = cscale(v[i], s);
}

// Finish Hessenberg column j: apply the previous Givens rotations, form the new
// one, rotate the right-hand side g and decide whether the cycle ends here.
__device__ void finish_column(KState& S, int j, int restart, int* skip_step, int rhs) {
  cpx<double>* col = S.H + (size_t)j * (kMaxRestart + 1);
  for (int i = 0; i <= j; ++i) col[i] = S.h[i];
  const double hn = S.hnext;
  for (int i = 0; i < j; ++i) {
    const cpx<double> a = col[i], b = col[i + 1];
    const cpx<double> c = S.cs[i], s = S.sn[i];
    // [conj(c) conj(s); -s c] applied to (a, b)
    col[i] = {c.re * a.re + c.im * a.im + s.re * b.re + s.im * b.im,
              c.re * a.im - c.im * a.re + s.re * b.im - s.im * b.re};
    col[i + 1] = {-(s.re * a.re - s.im * a.im) + (c.re * b.re - c.im * b.im),
                  -(s.re * a.im + s.im * a.re) + (c.re * b.im + c.im * b.re)};
  }
  const cpx<double> a = col[j];
  const double aa = sqrt(cabs2(a));
  const double den = sqrt(aa * aa + hn * hn);
  cpx<double> c, s;
  if (den == 0.0) { c = {1.0, 0.0}; s = {0.0, 0.0}; }
  else if (aa == 0.0) { c = {0.0, 0.0}; s = {1.0, 0.0}; }
  else { c = {a.re / den, a.im / den}; s = {hn / den, 0.0}; }
  S.cs[j] = c;
  S.sn[j] = s;
  col[j] = {den, 0.0};
  col[j + 1] = {0.0, 0.0};
  const cpx<double> gj = S.g[j];
  S.g[j] = {c.re * gj.re + c.im * gj.im, c.re * gj.im - c.im * gj.re};   // conj(c) g_j
  S.g[j + 1] = {-s.re * gj.re, -s.re * gj.im};
  S.k = j + 1;
  S.iters += 1;
  const double est = sqrt(cabs2(S.g[j + 1]));
  const bool breakdown = hn <= 1e-14 * sqrt(S.w2_first);
  if (est <= S.target || breakdown || j + 1 >= restart) skip_step[rhs] = 1;
}

// stage 1: projections h = V^H w and ||w||^2; a second projection is needed when
// more than half of ||w||^2 was removed (Kahan-Parlett / DGKS criterion).
// stage 2: the second projections are added to h.
__global__ __launch_bounds__(1024) void k_arnoldi_reduce(const cpx<double>* part, KState* state,
                                                         int* skip_step, int j, int stage, int restart) {
  __shared__ cpx<double> sums[kMaxRestart + 2];
  const int rhs = blockIdx.x;
  if (skip_step[rhs]) return;
  KState& S = state[rhs];
  if (stage == 2 && !S.reorth) return;
  reduce_slots(part, rhs, j + 2, sums);
  if (threadIdx.x != 0) return;
  double hh = 0.0;
  const double w2 = sums[j + 1].re;
  if (stage == 1) {
    for (int i = 0; i <= j; ++i) { S.h[i] = sums[i]; hh += cabs2(sums[i]); }
    S.w2_first = w2;
    const double p2 = w2 - hh;
    if (p2 > 0.5 * w2) {
      S.reorth = 0;
      S.hnext = sqrt(p2);
      finish_column(S, j, restart, skip_step, rhs);
    } else {
      S.reorth = 1;
    }
  } else {
    for (int i = 0; i <= j; ++i) {
      S.h2[i] = sums[i];
      S.h[i] = cadd(S.h[i], sums[i]);
      hh += cabs2(sums[i]);
    }
    const double p2 = w2 - hh;
    S.hnext = p2 > 0.0 ? sqrt(p2) : 0.0;
    finish_column(S, j, restart, skip_step, rhs);
  }
}

// stage 1 without reorthogonalisation: v_{j+1} = (w - V h) / h_{j+1,j}.
// stage 1 with: w <- w - V h (kept in place) and partial sums of V^H w, ||w||^2.
// stage 2: v_{j+1} = (w - V h2) / h_{j+1,j}.
__global__ __launch_bounds__(kRedThreads) void k_arnoldi_update(cpx<double>* __restrict__ V, size_t npts,
                                                                size_t vrs, const KState* __restrict__ state,
                                                                cpx<double>* __restrict__ part,
                                                                const int* __restrict__ skip_step, int j,
                                                                int stage) {
  __shared__ cpx<double> coef[kMaxRestart + 1];
  const int rhs = blockIdx.y;
  if (skip_step[rhs]) return;
  const KState& S = state[rhs];
  const int reorth = S.reorth;
  if (stage == 2 && !reorth) return;
  const bool final_pass = (stage == 2) || !reorth;
  for (int i = threadIdx.x; i <= kMaxRestart; i += blockDim.x)
    coef[i] = i > j ? cpx<double>{0.0, 0.0} : (stage == 1 ? S.h[i] : S.h2[i]);
  __syncthreads();
  const double inv = final_pass ? 1.0 / S.hnext : 1.0;
  cpx<double>* Vr = V + (size_t)rhs * vrs;
  cpx<double>* w = Vr + (size_t)(j + 1) * npts;
  const size_t stride = (size_t)kRedBlocks * kRedThreads;
  if (final_pass) {
    for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < npts; i += stride) {
      cpx<double> a = w[i];
      // groups of 8 basis vectors: their loads are independent and issued together
      for (int v0 = 0; v0 <= j; v0 += 8) {
        cpx<double> b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) b[u] = (v0 + u <= j) ? Vr[(size_t)(v0 + u) * npts + i] : cpx<double>{0.0, 0.0};
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const cpx<double> c = coef[v0 + u < kMaxRestart + 1 ? v0 + u : kMaxRestart];
          a.re -= c.re * b[u].re - c.im * b[u].im;
          a.im -= c.re * b[u].im + c.im * b[u].re;
        }
      }
      w[i] = cscale(a, inv);
    }
    return;
  }
  // reorthogonalisation path: update in place, then project again
  cpx<double>* pr = part + ((size_t)rhs * kRedBlocks + blockIdx.x) * kPartSlots;
  {
    cpx<double> nrm[1] = {{0.0, 0.0}};
    for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < npts; i += stride) {
      cpx<double> a = w[i];
      for (int v0 = 0; v0 <= j; v0 += 8) {
        cpx<double> b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) b[u] = (v0 + u <= j) ? Vr[(size_t)(v0 + u) * npts + i] : cpx<double>{0.0, 0.0};
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const cpx<double> c = coef[v0 + u < kMaxRestart + 1 ? v0 + u : kMaxRestart];
          a.re -= c.re * b[u].re - c.im * b[u].im;
          a.im -= c.re * b[u].im + c.im * b[u].re;
        }
      }
      w[i] = a;
      nrm[0].re += a.re * a.re + a.im * a.im;
    }
    block_reduce_write<1>(nrm, 1, pr + j + 1);
  }
  const int nvec = j + 1;
  for (int c0 = 0; c0 < nvec; c0 += kChunk) {
    const int cnt = nvec - c0 < kChunk ? nvec - c0 : kChunk;
    cpx<double> acc[kChunk];
#pragma unroll
    for (int v = 0; v < kChunk; ++v) acc[v] = {0.0, 0.0};
    for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < npts; i += stride) {
      const cpx<double> a = w[i];
#pragma unroll
      for (int v = 0; v < kChunk; ++v) {
        if (v < cnt) {
          const cpx<double> b = Vr[(size_t)(c0 + v) * npts + i];
          acc[v].re += b.re * a.re + b.im * a.im;
          acc[v].im += b.re * a.im - b.im * a.re;
        }
      }
    }
    block_reduce_write<kChunk>(acc, cnt, pr + c0);
  }
}

// y = R^{-1} g over the k finished columns (upper triangular back substitution).
__global__ void k_backsolve(KState* state, const int* done) {
  const int rhs = blockIdx.x;
  if (done[rhs] || threadIdx.x != 0) return;
  KState& S = state[rhs];
  const int k = S.k;
  for (int i = k - 1; i >= 0; --i) {
    cpx<double> s = S.g[i];
    for (int l = i + 1; l < k; ++l) {
      const cpx<double> r = S.H[(size_t)l * (kMaxRestart + 1) + i];
      s = csub(s, cmul(r, S.y[l]));
    }
    const cpx<double> d = S.H[(size_t)i * (kMaxRestart + 1) + i];
    const double dd = cabs2(d);
    S.y[i] = {(s.re * d.re + s.im * d.im) / dd, (s.im * d.re - s.re * d.im) / dd};
  }
}

// out = sum_{i<k} y_i v_i
__global__ __launch_bounds__(256) void k_lincomb(const cpx<double>* __restrict__ V, size_t npts, size_t vrs,
                                                 const KState* __restrict__ state, cpx<double>* __restrict__ out,
                                                 size_t out_rs, const int* __restrict__ done) {
  __shared__ cpx<double> y[kMaxRestart];
  const int rhs = blockIdx.y;
  if (done[rhs]) return;
  const KState& S = state[rhs];
  const int k = S.k;
  for (int i = threadIdx.x; i < k; i += blockDim.x) y[i] = S.y[i];
  __syncthreads();
  const cpx<double>* Vr = V + (size_t)rhs * vrs;
  cpx<double>* o = out + (size_t)rhs * out_rs;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < npts; i += (size_t)gridDim.x * 256) {
    cpx<double> a = {0.0, 0.0};
    for (int v0 = 0; v0 < k; v0 += 8) {
      cpx<double> b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = (v0 + u < k) ? Vr[(size_t)(v0 + u) * npts + i] : cpx<double>{0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const cpx<double> c = (v0 + u < k) ? y[v0 + u] : cpx<double>{0.0, 0.0};
        a.re += c.re * b[u].re - c.im * b[u].im;
        a.im += c.re * b[u].im + c.im * b[u].re;
      }
    }
    o[i] = a;
  }
}

__global__ void k_fill_zero(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

static unsigned stream_blocks(size_t npts) {
  size_t b = (npts + 255) / 256;
  return (unsigned)(b < 2048 ? (b == 0 ? 1 : b) : 2048);
}

hipError_t launch_dots(const KrylovArgs& a, const cpx<double>* w, size_t wrs, int nvec, const int* skip,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_dots, dim3(kRedBlocks, a.nrhs), dim3(kRedThreads), 0, st, a.V, a.npts, a.vrs, w, wrs,
                     nvec, a.part, skip);
  return hipGetLastError();
}

hipError_t launch_fnorm(const KrylovArgs& a, double rtol, hipStream_t st) {
  hipLaunchKernelGGL(k_fnorm, dim3(a.nrhs), dim3(1024), 0, st, a.part, a.state, a.done, rtol);
  return hipGetLastError();
}

hipError_t launch_cycle_start(const KrylovArgs& a, double rtol, hipStream_t st) {
  hipLaunchKernelGGL(k_cycle_start, dim3(a.nrhs), dim3(1024), 0, st, a.part, a.state, a.done, a.skip_step,
                     rtol);
  return hipGetLastError();
}

hipError_t launch_scale_v0(const KrylovArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_v0, dim3(stream_blocks(a.npts), a.nrhs), dim3(256), 0, st, a.V, a.npts, a.vrs,
                     a.state, a.done);
  return hipGetLastError();
}

hipError_t launch_arnoldi_reduce(const KrylovArgs& a, int j, int stage, hipStream_t st) {
  hipLaunchKernelGGL(k_arnoldi_reduce, dim3(a.nrhs), dim3(1024), 0, st, a.part, a.state, a.skip_step, j, stage,
                     a.restart);
  return hipGetLastError();
}

hipError_t launch_arnoldi_update(const KrylovArgs& a, int j, int stage, hipStream_t st) {
  hipLaunchKernelGGL(k_arnoldi_update, dim3(kRedBlocks, a.nrhs), dim3(kRedThreads), 0, st, a.V, a.npts, a.vrs,
                     a.state, a.part, a.skip_step, j, stage);
  return hipGetLastError();
}

hipError_t launch_backsolve(const KrylovArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_backsolve, dim3(a.nrhs), dim3(64), 0, st, a.state, a.done);
  return hipGetLastError();
}

hipError_t launch_lincomb(const KrylovArgs& a, cpx<double>* out, size_t out_rs, hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb, dim3(stream_blocks(a.npts), a.nrhs), dim3(256), 0, st, a.V, a.npts, a.vrs,
                     a.state, out, out_rs, a.done);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3(stream_blocks(n)), dim3(256), 0, st, (uint32_t*)p, n);
  return hipGetLastError();
}

}  // namespace hp
