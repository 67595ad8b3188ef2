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
#include <algorithm>
#include <mutex>
#include <type_traits>

#include <hip/hip_ext.h>

#include "hp_internal.h"

// Launch of a pass kernel; with timing events (tev non-null) through
// hipExtLaunchKernelGGL, which stores the kernel's own start and end times in
// tev[0] and tev[1] (no marker packets around it).
#define HP_PASS_LAUNCH(tev, kernel, grid, block, shm, st, ...)                                         \
  do {                                                                                                 \
    if ((tev) != nullptr)                                                                              \
      hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)(shm), st, (tev)[0], (tev)[1], 0, __VA_ARGS__); \
    else                                                                                               \
      hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);                                    \
  } while (0)

namespace hp {

template <typename R, typename S>
__device__ __forceinline__ cpx<R> cvt(cpx<S> a) {
  return {(R)a.re, (R)a.im};
}

// Rows (contiguous axis): G lines of length N per workgroup of 256 threads
// (one line per workgroup when a line needs 256 threads or more).
#ifndef HP_ROWC_THREADS
#define HP_ROWC_THREADS 64
#endif
#ifndef HP_PREFETCH_C
#define HP_PREFETCH_C 0
#endif
// mixed-radix column and combine passes gather each stage's twiddles into LDS at the
// start of a workgroup (consecutive butterflies then read consecutive entries); pass A
// reads the line's table from global memory (one transform per workgroup)
#ifndef HP_GEN_LDS_TW
#define HP_GEN_LDS_TW 1
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
template <typename R, int N, int MAXT, int SEG = 64, int EE = elems_per_thread<R>(N)>
struct ColCfg {
  static constexpr int E = EE;
  static constexpr int T = N / E;
  static constexpr int TC0 = SEG / (2 * (int)sizeof(R));
  static constexpr int THR0 = TC0 * T < 256 ? 256 : TC0 * T;
  static constexpr int THREADS = THR0 > MAXT ? MAXT : THR0;
  static constexpr int TC = THREADS / T;
  static constexpr int LDS = (N > E) ? TC * lds_elems_e<E>(N) : 1;
};
#ifndef HP_SYM_MAXT
#define HP_SYM_MAXT 512
#endif
#ifndef HP_SYM_SEG
#define HP_SYM_SEG 32
#endif
// elements per thread of the symbol pass (it keeps the forward spectrum and the
// symbol argument in registers besides the transform, so it may use fewer)
#ifndef HP_SYM_E64
#define HP_SYM_E64 HP_E64
#endif
#ifndef HP_SYM_E32
#define HP_SYM_E32 HP_E32
#endif
template <typename R>
constexpr int sym_elems(int n) {
  return n < (sizeof(R) == 8 ? HP_SYM_E64 : HP_SYM_E32) ? n : (sizeof(R) == 8 ? HP_SYM_E64 : HP_SYM_E32);
}
template <typename R, int N>
using SymCfg = ColCfg<R, N, HP_SYM_MAXT, HP_SYM_SEG, sym_elems<R>(N)>;
template <typename R, int N, int MODE>
using ColsCfg = std::conditional_t<MODE == 1, SymCfg<R, N>, ColCfg<R, N, 1024>>;
#ifndef HP_XCD_REMAP
#define HP_XCD_REMAP 1
#endif
// Pass C with one row per wavefront (k_comb_wave) for the precisions in
// HP_WAVE_COMB (bit 0: FP32 lines, bit 1: FP64 lines).  FP32 1024-point rows:
// 56.9 -> 53-54 us per 1024^2 combine; FP64 1024-point rows need more than 256
// registers at 16 elements per lane (spills, 64 -> 131 us), so they keep the
// two-wavefront rows of k_rows_combine.
#ifndef HP_WAVE_COMB
#define HP_WAVE_COMB 1
#endif

// FP64 lines of 1024 points (stages 8, 8, 8, 2) and, in the row passes, of 2048
// (8, 8, 8, 4) take the exchange before their last stage through lanes
// (v_permlane32_swap / v_permlane16_swap) instead of LDS and two barriers
// (lane_exchange_kind and Stage in the FFT engine).  The threads that trade must
// share a wavefront at the lanes Stage expects, so these lines number their threads
// differently.  Measured and left off: the 2048-point symbol pass (741 -> 831 us:
// its column tiles' loads spread over four row groups per wavefront) and the FP32
// lines of 1024 points (16, 16, 4), whose LDS exchanges need only wavefront
// barriers (1024^2 mixed combine 55.7 -> 63.0 us).
#ifndef HP_LANE_SWAP
#define HP_LANE_SWAP 1
#endif
template <typename R, int N>
constexpr int rows_swap() {
  constexpr int E = elems_per_thread<R>(N), T = N / E, K = lane_exchange_kind<N, E>();
  if (!HP_LANE_SWAP || sizeof(R) != 8) return 0;
  return ((T == 128 && K == 2) || (T == 256 && K == 4)) ? 32 : 0;
}
// j of the thread with index tl within its line: 128 threads, j ^ 64 at lane ^ 32;
// 256 threads, j >> 6 in lane bits 4-5
template <typename R, int N>
__device__ __forceinline__ int rows_thread(int tl) {
  constexpr int T = N / elems_per_thread<R>(N);
  const int lane = tl & 63;
  if constexpr (rows_swap<R, N>() != 0 && T == 128) return (lane & 31) | (((tl >> 6) & 1) << 5) | ((lane >> 5) << 6);
  else if constexpr (rows_swap<R, N>() != 0 && T == 256) return ((lane >> 4) << 6) | (((tl >> 6) & 3) << 4) | (lane & 15);
  else return tl;
}

// ---------------------------------------------------------------- pass A
// Pass bodies take their workgroup's indices and LDS as arguments, so that the
// grouped launches (several plans, several line lengths in one launch) run the
// same code as the single-plan kernels.
template <typename R, typename TI, int N>
__device__ __forceinline__ void rows_fwd_body(const cpx<TI>* __restrict__ in, cpx<R>* __restrict__ out, int rows,
                                              size_t in_rs, size_t out_rs, const cpx<R>* __restrict__ tw, int bx,
                                              int rhs, cpx<R>* lds) {
  using C = RowCfg<R, N>;
  constexpr int SWP = rows_swap<R, N>();
  const int g = threadIdx.x / C::T, j = rows_thread<R, N>((int)threadIdx.x % C::T);
  const int row = bx * C::G + g;
  const bool act = row < rows;
  const cpx<TI>* src = in + (size_t)rhs * in_rs + (size_t)row * N;
  cpx<R> x[C::E];
#pragma unroll
  for (int s = 0; s < C::E; ++s) x[s] = act ? cvt<R>(src[j + C::T * s]) : cpx<R>{0, 0};
  fft_e<R, N, C::E, -1, true, 1, false, SWP>(x, lds + g * lds_elems<R>(N), j, tw);
  if (act) {
    cpx<R>* dst = out + (size_t)rhs * out_rs + (size_t)row * N;
#pragma unroll
    for (int s = 0; s < C::E; ++s) dst[j + C::T * s] = x[s];
  }
}

template <typename R, typename TI, int N>
__global__ __launch_bounds__((RowCfg<R, N>::THREADS)) void k_rows_fwd(const cpx<TI>* __restrict__ in,
                                                                  cpx<R>* __restrict__ out, int rows,
                                                                  size_t in_rs, size_t out_rs,
                                                                  const cpx<R>* __restrict__ tw,
                                                                  const int* __restrict__ skip) {
  __shared__ cpx<R> lds[RowCfg<R, N>::LDS];
  const int rhs = blockIdx.y;
  if (skip != nullptr && skip[rhs] != 0) return;
  rows_fwd_body<R, TI, N>(in, out, rows, in_rs, out_rs, tw, blockIdx.x, rhs, lds);
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

// The column pass of one workgroup: (bx, by, bz) and (gx, gy) stand for blockIdx
// and gridDim.
template <typename R, int N, int MODE>
constexpr int cols_smask_words() {
  return MODE == 1 ? kMaxNodes * ColsCfg<R, N, MODE>::T : 1;
}

// The symbol pass takes the same lane exchange for its 1024-point FP64 columns
// (two columns of 128 threads per workgroup).
template <typename R, int N, int MODE>
constexpr int cols_swap() {
  using C = ColsCfg<R, N, MODE>;
  return HP_LANE_SWAP && MODE == 1 && sizeof(R) == 8 && lane_exchange_kind<N, C::E>() == 2 && C::T == 128 &&
                 C::TC == 2 && C::THREADS == 256
             ? 32
             : 0;
}

template <typename R, typename TI, int N, int DIR, int MODE>
__device__ __forceinline__ void cols_body(
    const cpx<TI>* __restrict__ in, cpx<R>* __restrict__ out, int S, int nfields, size_t in_rs,
    size_t out_rs, size_t in_fs, size_t out_fs, const cpx<R>* __restrict__ tw,
    const int* __restrict__ skip, const double* __restrict__ lam_ax, const double* __restrict__ lam_in,
    const NodeConst* __restrict__ nodes, int K, double scale, const uint16_t* __restrict__ store_mask,
    const uint8_t* __restrict__ slab_need, int bx, int by, int bz, int gx, int gy, cpx<R>* lds, uint16_t* smask) {
  using C = ColsCfg<R, N, MODE>;
  constexpr int SWP = cols_swap<R, N, MODE>();
  const int z = bz;
  const int rhs = (MODE == 0) ? z / nfields : z;
  const int fld = (MODE == 0) ? z % nfields : 0;
  if (skip != nullptr && skip[rhs] != 0) return;
  // plain passes over node fields: slabs whose points never use this node are skipped
  if (MODE == 0 && slab_need != nullptr && slab_need[(size_t)fld * gy + by] == 0) return;
  // With the lane exchange threads j and j ^ 64 of a column sit at lanes l and l ^ 32
  // of one wavefront: lane = (j >> 6) << 5 | (j & 15) << 1 | g, wavefront (j >> 4) & 3.
  const int lane = threadIdx.x & 63;
  const int g = SWP ? (lane & 1) : (int)threadIdx.x % C::TC;
  const int j = SWP ? (((lane >> 1) & 15) | ((int)(threadIdx.x >> 6) << 4) | ((lane >> 5) << 6))
                    : (int)threadIdx.x / C::TC;
  // Workgroups are dispatched round-robin over the 8 XCDs (each with its own
  // L2).  Give the workgroups of one XCD consecutive column tiles so that tiles
  // sharing cache lines meet in the same L2.
  int tile = bx;
#if HP_XCD_REMAP
  if ((gx & 7) == 0) tile = (bx & 7) * (gx >> 3) + (bx >> 3);
#endif
  const int c = tile * C::TC + g;
  const bool act = c < S;
  // MODE 0: by is the outer (slab) index.  MODE 1 (outer = 1): by is the node
  // group; small grids split the nodes over several workgroups per column tile
  // (each redoes the forward transform) so that the launch fills the GPU.
  const size_t obase = (MODE == 0 ? (size_t)by * N * S : 0) + c;
  const cpx<TI>* src = in + (size_t)rhs * in_rs + (size_t)fld * in_fs + obase;
  cpx<R>* lg = lds + g;   // the TC columns are interleaved in LDS
  // Symbol pass: the store masks of all nodes are staged in LDS up front, so that
  // the node loop issues no global load (waiting for one would also wait for the
  // previous node's stores: vector memory operations retire in order).
  if constexpr (MODE == 1) {
    for (int i = threadIdx.x; i < K * C::T; i += C::THREADS) smask[i] = store_mask[i];
    __syncthreads();
  }
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
    fft_e<R, N, C::E, -1, false, C::TC, false, SWP>(x, lg, j, tw);
    cpx<R> vh[C::E];
    double lam[C::E];
    const double lc = act ? lam_in[c] : 0.0;
#pragma unroll
    for (int s = 0; s < C::E; ++s) {
      vh[s] = x[s];
      lam[s] = lam_ax[j + C::T * s] + lc;
    }
    cpx<R>* dst = out + (size_t)rhs * out_rs + obase;
    const int n_lo = (int)(((long)by * K) / gy), n_hi = (int)(((long)(by + 1) * K) / gy);
    for (int n = n_lo; n < n_hi; ++n) {
      symbol_mul<R, C::E>(vh, x, lam, nodes[n], scale);
      fft_e<R, N, C::E, +1, false, C::TC, false, SWP>(x, lg, j, tw);
      // bit s: some point of axis-0 index j + T*s uses node n (else the row is never read)
      const uint32_t m = act ? (uint32_t)smask[n * C::T + j] : 0u;
#pragma unroll
      for (int s = 0; s < C::E; ++s)
        if ((m >> s) & 1u) dst[(size_t)n * out_fs + (size_t)(j + C::T * s) * S] = x[s];
    }
  }
}

template <typename R, typename TI, int N, int DIR, int MODE>
__global__ __launch_bounds__((ColsCfg<R, N, MODE>::THREADS)) void k_cols(
    const cpx<TI>* __restrict__ in, cpx<R>* __restrict__ out, int S, int nfields, size_t in_rs,
    size_t out_rs, size_t in_fs, size_t out_fs, const cpx<R>* __restrict__ tw,
    const int* __restrict__ skip, const double* __restrict__ lam_ax, const double* __restrict__ lam_in,
    const NodeConst* __restrict__ nodes, int K, double scale, const uint16_t* __restrict__ store_mask,
    const uint8_t* __restrict__ slab_need) {
  __shared__ cpx<R> lds[ColsCfg<R, N, MODE>::LDS];
  __shared__ uint16_t smask[cols_smask_words<R, N, MODE>()];
  cols_body<R, TI, N, DIR, MODE>(in, out, S, nfields, in_rs, out_rs, in_fs, out_fs, tw, skip, lam_ax, lam_in, nodes,
                                 K, scale, store_mask, slab_need, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x,
                                 gridDim.y, lds, smask);
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

// Interpolation modes of the combine: piecewise linear along Re gamma (the
// paper's), piecewise Lagrange of degree >= 2 along the real axis, and bilinear in
// (c, a) (one damping node axis; no layer).
enum InterpMode { kInterpLinear = 0, kInterpLagrange = 1, kInterpBilinear = 2 };

// Per-point record for the combine: `ab` packs nodes A, B (piecewise linear:
// weights 1-t, t) or, for a real-axis point under Lagrange interpolation of degree
// ord >= 2, the first node A of its ord+1-node stencil and a flag; `tt` holds t,
// or the point's speed x for the Lagrange weights.  Bilinear: `ab` packs the four
// nodes (s, r), (s+1, r), (s, r+1), (s+1, r+1) of node index m + M r, `tt` and `uu`
// the fractions along c and along a.  lag: the table of CombineArgs.
template <typename R, int IM>
__device__ __forceinline__ void interp_record(double pv, double pa, int M, int Mt, int mo, int Ma, int ord,
                                              const double* lag, int& ab, R& tt, R& uu) {
  int A = -1, B = -1;
  double t = 0.0;
  decode_pos(pv, M, Mt, mo, A, B, t);
  if (IM == kInterpBilinear) {
    int r = (int)pa;
    if (r > Ma - 2) r = Ma - 2;
    if (r < 0) r = 0;
    const double u = pa - (double)r;
    A += M * r;
    B += M * r;
    ab = A | (B << 8) | ((A + M) << 16) | ((B + M) << 24);
    tt = (R)t;
    uu = (R)u;
  } else if (IM == kInterpLagrange && pv >= 0.0 && M > 1) {
    int a = A - (ord - 1) / 2;
    a = a < 0 ? 0 : (a > M - 1 - ord ? M - 1 - ord : a);
    ab = a | (1 << 16);
    tt = (R)(lag[A] + t * (lag[A + 1] - lag[A]));
  } else {
    ab = (A & 0xff) | ((B & 0xff) << 8);
    tt = (R)t;
  }
}

// Weight of node n at a point with record (ab, tt, uu).
template <typename R, int IM>
__device__ __forceinline__ R interp_weight(int ab, R tt, R uu, int n, int ord, const double* lag) {
  const int A = ab & 0xff;
  if (IM == kInterpBilinear) {
    const int B = (ab >> 8) & 0xff, Cn = (ab >> 16) & 0xff, D = (ab >> 24) & 0xff;
    const R lo = (R)1 - uu;
    return (A == n ? ((R)1 - tt) * lo : (R)0) + (B == n ? tt * lo : (R)0) + (Cn == n ? ((R)1 - tt) * uu : (R)0) +
           (D == n ? tt * uu : (R)0);
  }
  if (IM == kInterpLagrange && (ab >> 16)) {
    if (n < A || n > A + ord) return (R)0;
    R w = (R)lag[kMaxNodes + 4 * n + (n - A)];
    for (int k = A; k <= A + ord; ++k)
      if (k != n) w *= tt - (R)lag[k];
    return w;
  }
  const int B = (ab >> 8) & 0xff;
  return (A == n ? (R)1 - tt : (R)0) + (B == n ? tt : (R)0);
}

// NS > 1 (lines of at most one wavefront, few rows): NS wavefronts share the
// workgroup's rows, wavefront s taking every NS-th node the rows use, and their
// partial sums meet in LDS at the end; the node loop is NS times shorter and the
// chip holds NS times more wavefronts.
template <typename R, int N>
constexpr bool combine_splits_fit() {
  return CombCfg<R, N>::T <= 64 && N >= 128;
}
constexpr int kCombineSplits = 4;

template <typename R, int N, int NS>
constexpr int combine_lds_elems() {
  using C = CombCfg<R, N>;
  constexpr int XCH = NS * C::LDS, RED = (NS - 1) * C::G * N;
  return XCH > RED ? XCH : RED;
}

// bx: the row group (blockIdx.x of the single-plan kernel)
template <typename R, typename TO, int N, bool ACC, int IM, int NS>
__device__ __forceinline__ void rows_combine_body(
    const cpx<R>* __restrict__ fields, size_t fs, size_t frs, const double* __restrict__ pos,
    const uint64_t* __restrict__ grpmask, const uint64_t* __restrict__ rowmask, cpx<TO>* __restrict__ out,
    size_t out_rs, int rows, int K, int M, int Mt, int mo, const cpx<R>* __restrict__ tw,
    const int* __restrict__ skip, int ord, const double* __restrict__ lag, const double* __restrict__ posa, int Ma,
    int bx, int rhs, cpx<R>* lds, double* slag) {
  using C = CombCfg<R, N>;
  static_assert(NS == 1 || combine_splits_fit<R, N>(), "node splits need transforms within one wavefront");
  constexpr bool LAG = IM == kInterpLagrange;
  if (skip != nullptr && skip[rhs] != 0) return;
  if constexpr (LAG) {
    for (int i = threadIdx.x; i < kLagTable; i += C::THREADS * NS) slag[i] = lag[i];
    __syncthreads();
  }
  constexpr int SWP = NS == 1 ? rows_swap<R, N>() : 0;
  const int sp = NS > 1 ? (int)threadIdx.x / C::THREADS : 0;
  const int tl = NS > 1 ? (int)threadIdx.x % C::THREADS : (int)threadIdx.x;
  const int g = tl / C::T, j = SWP ? rows_thread<R, N>(tl % C::T) : tl % C::T;
  const int row = bx * C::G + g;
  const bool act = row < rows;
  const size_t rbase = (size_t)row * N;
  int ab[C::E];
  R tt[C::E], uu[C::E];
  cpx<R> acc[C::E];
#pragma unroll
  for (int s = 0; s < C::E; ++s) {
    ab[s] = 0xffff;
    tt[s] = (R)0;
    uu[s] = (R)0;
    if (act) {
      const size_t pi = rbase + j + C::T * s;
      interp_record<R, IM>(pos[pi], IM == kInterpBilinear ? posa[pi] : 0.0, M, Mt, mo, Ma, ord, slag, ab[s], tt[s],
                           uu[s]);
    }
    acc[s] = {0, 0};
  }
  const uint64_t mask = grpmask[bx];
  const uint64_t rmask = act ? rowmask[row] : 0ull;
  const cpx<R>* fr = fields + (size_t)rhs * frs + rbase;
  cpx<R>* lg = lds + (sp * C::G + g) * lds_elems<R>(N);
  // Nodes no point of this group uses are skipped; rows that do not use a node
  // read zeros (pass B did not write them).  The next used node's row is loaded
  // while the current one is transformed.
  auto next_node = [&](int n) {
    while (n < K && ((mask >> n) & 1ull) == 0) ++n;
    return n;
  };
  // the node after the next NS - 1 used ones (this split's next node)
  auto split_next = [&](int n) {
    for (int q = 0; q < NS && n < K; ++q) n = next_node(n + 1);
    return n;
  };
  cpx<R> nx[C::E];
  int n = next_node(0);
  for (int q = 0; q < sp && n < K; ++q) n = next_node(n + 1);
  if (!HP_PREFETCH_C && n < K) {
    // loaded at the top of the loop instead
  } else if (n < K) {
    const bool ld = ((rmask >> n) & 1ull) != 0;
#pragma unroll
    for (int s = 0; s < C::E; ++s) nx[s] = ld ? fr[(size_t)n * fs + j + C::T * s] : cpx<R>{0, 0};
  }
  for (; n < K;) {
    cpx<R> x[C::E];
    const int n2 = NS > 1 ? split_next(n) : next_node(n + 1);
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
    fft_e<R, N, C::E, +1, true, 1, false, SWP>(x, lg, j, tw);
#pragma unroll
    for (int s = 0; s < C::E; ++s) {
      const R w = interp_weight<R, IM>(ab[s], tt[s], uu[s], n, ord, slag);
      acc[s].re += w * x[s].re;
      acc[s].im += w * x[s].im;
    }
    n = n2;
  }
  if constexpr (NS > 1) {   // partial sums of the splits, added by split 0 in a fixed order
    __syncthreads();        // every split is done with its exchange area
    if (sp > 0) {
#pragma unroll
      for (int s = 0; s < C::E; ++s) lds[((sp - 1) * C::G + g) * N + j + C::T * s] = acc[s];
    }
    __syncthreads();
    if (sp > 0) return;
    for (int q = 1; q < NS; ++q) {
#pragma unroll
      for (int s = 0; s < C::E; ++s) {
        const cpx<R> o = lds[((q - 1) * C::G + g) * N + j + C::T * s];
        acc[s].re += o.re;
        acc[s].im += o.im;
      }
    }
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

template <typename R, typename TO, int N, bool ACC, int IM, int NS = 1>
__global__ __launch_bounds__((CombCfg<R, N>::THREADS * NS)) void k_rows_combine(
    const cpx<R>* __restrict__ fields, size_t fs, size_t frs, const double* __restrict__ pos,
    const uint64_t* __restrict__ grpmask, const uint64_t* __restrict__ rowmask, cpx<TO>* __restrict__ out,
    size_t out_rs, int rows, int K, int M, int Mt, int mo, const cpx<R>* __restrict__ tw,
    const int* __restrict__ skip, int ord, const double* __restrict__ lag, const double* __restrict__ posa, int Ma) {
  __shared__ cpx<R> lds[combine_lds_elems<R, N, NS>()];
  __shared__ double slag[IM == kInterpLagrange ? kLagTable : 1];
  rows_combine_body<R, TO, N, ACC, IM, NS>(fields, fs, frs, pos, grpmask, rowmask, out, out_rs, rows, K, M, Mt, mo, tw,
                                           skip, ord, lag, posa, Ma, blockIdx.x, blockIdx.y, lds, slag);
}

// ---------------------------------------------------------------- wave-resident lines
// A line of N = 64 E points held by one wavefront, E elements per lane (E = 16 at
// N = 1024): every exchange of its transform stays inside the wavefront, so the
// transform needs no workgroup barrier and each wavefront runs at its own pace;
// with radix-E stages a 1024-point line takes two exchanges instead of three.
// At E = 16 the twiddles of all stages would take more registers than the line
// itself if the compiler kept them live across a node loop (they are loop
// invariant), so each stage reads its own again from the cache (fft_e with
// RELOAD).
template <typename R, int N>
struct WaveLine {
  static constexpr int E = N / 64;
  static constexpr int LDS = lds_elems_e<E>(N);
};
template <typename R, int N>
constexpr bool wave_line_fits() {
  // lines of one full wavefront with at most 16 elements per lane
  return N >= 256 && N / 64 <= 16;
}
constexpr int kWaveRows = 4;   // rows (one per wavefront) per workgroup of the wave combine

// Pass C with one row per wavefront: inverse transform of each node row the row
// uses (its own node list, not its workgroup's) and the weighted sum; loads and
// stores of a wavefront cover 64 E consecutive elements.
// WR rows per workgroup (one per wavefront); bx: the workgroup's row block
template <typename R, typename TO, int N, bool ACC, int IM, int WR>
__device__ __forceinline__ void comb_wave_body(
    const cpx<R>* __restrict__ fields, size_t fs, size_t frs, const double* __restrict__ pos,
    const uint64_t* __restrict__ rowmask, cpx<TO>* __restrict__ out, size_t out_rs, int rows, int M, int Mt,
    int mo, const cpx<R>* tw, const int* __restrict__ skip, int ord, const double* __restrict__ lag,
    const double* __restrict__ posa, int Ma, int bx, int rhs, cpx<R>* lds, double* slag) {
  constexpr int E = WaveLine<R, N>::E;
  constexpr bool LAG = IM == kInterpLagrange;
  if (skip != nullptr && skip[rhs] != 0) return;
  if constexpr (LAG) {
    for (int i = threadIdx.x; i < kLagTable; i += 64 * WR) slag[i] = lag[i];
    __syncthreads();
  }
  const int wv = (int)threadIdx.x / 64, j = (int)threadIdx.x % 64;
  const int row = bx * WR + wv;
  if (row >= rows) return;   // no workgroup barrier follows
  const size_t rbase = (size_t)row * N;
  int ab[E];
  R tt[E], uu[E];
  cpx<R> acc[E];
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const size_t pi = rbase + j + 64 * s;
    uu[s] = (R)0;
    interp_record<R, IM>(pos[pi], IM == kInterpBilinear ? posa[pi] : 0.0, M, Mt, mo, Ma, ord, slag, ab[s], tt[s],
                         uu[s]);
    acc[s] = {0, 0};
  }
  cpx<R>* lw = lds + wv * WaveLine<R, N>::LDS;
  const cpx<R>* fr = fields + (size_t)rhs * frs + rbase;
  uint64_t left = rowmask[row];
  while (left != 0) {
    const int n = __builtin_ctzll(left);
    left &= left - 1;
    cpx<R> x[E];
#pragma unroll
    for (int s = 0; s < E; ++s) x[s] = fr[(size_t)n * fs + j + 64 * s];
    fft_e<R, N, E, +1, true, 1, true>(x, lw, j, tw);
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const R w = interp_weight<R, IM>(ab[s], tt[s], uu[s], n, ord, slag);
      acc[s].re += w * x[s].re;
      acc[s].im += w * x[s].im;
    }
  }
  cpx<TO>* dst = out + (size_t)rhs * out_rs + rbase;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    if constexpr (ACC) {
      cpx<TO> o = dst[j + 64 * s];
      dst[j + 64 * s] = {o.re + (TO)acc[s].re, o.im + (TO)acc[s].im};
    } else {
      dst[j + 64 * s] = cvt<TO>(acc[s]);
    }
  }
}

template <typename R, typename TO, int N, bool ACC, int IM>
__global__ __launch_bounds__(64 * kWaveRows, 2) void k_comb_wave(
    const cpx<R>* __restrict__ fields, size_t fs, size_t frs, const double* __restrict__ pos,
    const uint64_t* __restrict__ rowmask, cpx<TO>* __restrict__ out, size_t out_rs, int rows, int M, int Mt,
    int mo, const cpx<R>* tw, const int* __restrict__ skip, int ord, const double* __restrict__ lag,
    const double* __restrict__ posa, int Ma) {
  __shared__ cpx<R> lds[kWaveRows * WaveLine<R, N>::LDS];
  __shared__ double slag[IM == kInterpLagrange ? kLagTable : 1];
  comb_wave_body<R, TO, N, ACC, IM, kWaveRows>(fields, fs, frs, pos, rowmask, out, out_rs, rows, M, Mt, mo, tw, skip,
                                               ord, lag, posa, Ma, blockIdx.x, blockIdx.y, lds, slag);
}

// ---------------------------------------------------------------- mixed-radix lines
// Line lengths N = 2^a 3^b 5^c that are not powers of two (the grids of Example 1,
// Section 5.1).  One line per workgroup (or tc interleaved lines), held in LDS
// (dynamic shared memory) and transformed by Stockham stages whose radix is any
// product of 2, 3 and 5 up to 16 (a 2400-point line takes three stages, 16, 15
// and 10), each stage's DFT done in registers as two passes of radix 2, 3, 4 or 5
// with fixed roots between them.  In a stage of radix R thread t handles
// butterflies t, t + T, ... of the N/R (at most 16/R of them, which the host's
// choice of T guarantees) and keeps their outputs in registers until every thread
// has read its inputs.  Element p of a line sits at LDS slot p + p/16 (one pad per
// 16 elements), which spreads the strided writes of the early stages over the banks.

#ifndef HP_GEN_PAD
#define HP_GEN_PAD 1
#endif
__host__ __device__ __forceinline__ int gpos(int p) { return HP_GEN_PAD ? p + (p >> 4) : p; }
// LDS slots a line of n elements takes
__host__ __device__ __forceinline__ size_t gen_line_slots(int n) { return (size_t)gpos(n - 1) + 1; }

// cos and sin of 2 pi m / r, evaluated at compile time for the butterflies' fixed
// roots: the angle is reduced to [0, pi/4] by the octant symmetries (exactly, in
// integers), then summed as a Taylor series.
constexpr double kPiD = 3.14159265358979323846;
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k < 14; ++k) { t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0)); s += t; }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 14; ++k) { t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k)); s += t; }
  return s;
}
// angle 2 pi m / r with 0 <= m <= r/8 (at most pi/4)
constexpr void small_cs(long m, long r, double& c, double& s) {
  const double x = 2.0 * kPiD * (double)m / (double)r;
  c = taylor_cos(x);
  s = taylor_sin(x);
}
constexpr void root_cs(long m, long r, double& c, double& s) {
  m %= r;
  double sg = 1.0;
  if (2 * m > r) { m = r - m; sg = -1.0; }           // sin(2 pi - x) = -sin x
  double cg = 1.0;                                   // now x in [0, pi]
  if (4 * m > r) { m = r - 2 * m; cg = -1.0; r *= 2; }  // x -> pi - x: cos flips; m/r -> (r/2 - m)/r
  // now x = 2 pi m / r in [0, pi/2]
  double cc = 0.0, ss = 0.0;
  if (8 * m > r) {                                   // x -> pi/2 - x swaps cos and sin
    small_cs(r - 4 * m, 4 * r, ss, cc);
  } else {
    small_cs(m, r, cc, ss);
  }
  c = cg * cc;
  s = sg * ss;
}
template <int RAD>
struct RootTab {
  double c[RAD], s[RAD];
};
template <int RAD>
constexpr RootTab<RAD> make_roots() {
  RootTab<RAD> t{};
  for (int m = 0; m < RAD; ++m) root_cs(m, RAD, t.c[m], t.s[m]);
  return t;
}
template <int RAD>
constexpr RootTab<RAD> kRoots = make_roots<RAD>();

// x exp(DIR 2 pi i m / RAD) for a fixed m (the quarter turns without multiplies)
template <typename R, int RAD, int DIR>
__device__ __forceinline__ cpx<R> mul_root(cpx<R> x, int m) {
  m %= RAD;
  if (m == 0) return x;
  if (2 * m == RAD) return {-x.re, -x.im};
  if (4 * m == RAD) return DIR > 0 ? cpx<R>{-x.im, x.re} : cpx<R>{x.im, -x.re};
  if (4 * m == 3 * RAD) return DIR > 0 ? cpx<R>{x.im, -x.re} : cpx<R>{-x.im, x.re};
  const R c = (R)kRoots<RAD>.c[m], sn = (R)(DIR * kRoots<RAD>.s[m]);
  return {x.re * c - x.im * sn, x.re * sn + x.im * c};
}

// DFTs of length 2, 3, 4 and 5 in place: out[k] = sum_t v[t] exp(DIR 2 pi i t k / RAD),
// with the symmetric pairs of terms combined.
template <typename R, int DIR>
__device__ __forceinline__ void dft2(cpx<R>& a, cpx<R>& b) {
  const cpx<R> s = cadd(a, b), d = csub(a, b);
  a = s;
  b = d;
}
template <typename R, int DIR>
__device__ __forceinline__ cpx<R> times_dir_i(cpx<R> x) {   // DIR i x
  return DIR > 0 ? cpx<R>{-x.im, x.re} : cpx<R>{x.im, -x.re};
}
template <typename R, int RAD, int DIR>
__device__ __forceinline__ void dft_prime(cpx<R> (&v)[RAD]) {
  if constexpr (RAD == 2) {
    dft2<R, DIR>(v[0], v[1]);
  } else if constexpr (RAD == 3) {
    constexpr double s3 = 0.86602540378443864676;   // sin(2 pi / 3)
    const cpx<R> a = cadd(v[1], v[2]);
    const cpx<R> d = csub(v[1], v[2]);
    const cpx<R> m = {v[0].re - (R)0.5 * a.re, v[0].im - (R)0.5 * a.im};
    const cpx<R> j = times_dir_i<R, DIR>(cpx<R>{(R)s3 * d.re, (R)s3 * d.im});
    v[0] = cadd(v[0], a);
    v[1] = cadd(m, j);
    v[2] = csub(m, j);
  } else if constexpr (RAD == 4) {
    const cpx<R> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const cpx<R> s13 = cadd(v[1], v[3]), d13 = times_dir_i<R, DIR>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  } else {
    static_assert(RAD == 5, "radix 2, 3, 4 or 5");
    constexpr double c1 = 0.30901699437494742410, s1 = 0.95105651629515357212;   // 2 pi / 5
    constexpr double c2 = -0.80901699437494742410, s2 = 0.58778525229247312917;  // 4 pi / 5
    const cpx<R> a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const cpx<R> a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const cpx<R> m1 = {v[0].re + (R)c1 * a1.re + (R)c2 * a2.re, v[0].im + (R)c1 * a1.im + (R)c2 * a2.im};
    const cpx<R> m2 = {v[0].re + (R)c2 * a1.re + (R)c1 * a2.re, v[0].im + (R)c2 * a1.im + (R)c1 * a2.im};
    const cpx<R> j1 = times_dir_i<R, DIR>(cpx<R>{(R)s1 * b1.re + (R)s2 * b2.re, (R)s1 * b1.im + (R)s2 * b2.im});
    const cpx<R> j2 = times_dir_i<R, DIR>(cpx<R>{(R)s2 * b1.re - (R)s1 * b2.re, (R)s2 * b1.im - (R)s1 * b2.im});
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(m1, j1);
    v[4] = csub(m1, j1);
    v[2] = cadd(m2, j2);
    v[3] = csub(m2, j2);
  }
}

// first factor of a stage radix: the DFT of length RAD = F·(RAD/F) runs as RAD/F
// DFTs of length F, fixed roots, then F DFTs of length RAD/F
constexpr int radix_first(int r) { return r % 5 == 0 ? 5 : r % 4 == 0 ? 4 : r % 3 == 0 ? 3 : 2; }

template <typename R, int RAD, int DIR>
__device__ __forceinline__ void dft_radix(cpx<R> (&v)[RAD]) {
  constexpr int F = radix_first(RAD), G = RAD / F;
  if constexpr (G == 1) {
    dft_prime<R, RAD, DIR>(v);
  } else {
    // input index t = tf G + tg, output index kf + F kg
    cpx<R> a[G][F];
#pragma unroll
    for (int tg = 0; tg < G; ++tg) {
      cpx<R> u[F];
#pragma unroll
      for (int tf = 0; tf < F; ++tf) u[tf] = v[tf * G + tg];
      dft_prime<R, F, DIR>(u);
#pragma unroll
      for (int kf = 0; kf < F; ++kf) a[tg][kf] = mul_root<R, RAD, DIR>(u[kf], tg * kf);
    }
#pragma unroll
    for (int kf = 0; kf < F; ++kf) {
      cpx<R> u[G];
#pragma unroll
      for (int tg = 0; tg < G; ++tg) u[tg] = a[tg][kf];
      dft_radix<R, G, DIR>(u);
#pragma unroll
      for (int kg = 0; kg < G; ++kg) v[kf + F * kg] = u[kg];
    }
  }
}

// One Stockham stage of radix RAD over the line in buf (element p at
// buf[gpos(p) << lg]) after ns = the product of the earlier radices.  Twiddles:
// with ST, tw holds this stage's table, entry (t - 1) ns + k = exp(-2 pi i k t /
// (ns RAD)) (consecutive k for consecutive butterflies); else tw is the line's
// table exp(-2 pi i j / n).  Indices advance by additions (no integer multiplies
// per element).
template <typename R, int RAD, int DIR, bool ST, int SMAX>
__device__ void gen_stage(cpx<R>* buf, int lg, int n, int ns, const cpx<R>* __restrict__ tw, int tid, int nthr) {
  constexpr int MB = SMAX / RAD;
  const int nb = n / RAD;
  const int step = n / (ns * RAD);
  cpx<R> o[MB][RAD];
  int kk[MB];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = tid + i * nthr;
    kk[i] = 0;
    if (b < nb) {
      const int k = ns > 1 ? b % ns : 0;
      kk[i] = k;
      int p = b;
#pragma unroll
      for (int t = 0; t < RAD; ++t, p += nb) o[i][t] = buf[gpos(p) << lg];
      if (ns > 1) {
        const int dq = ST ? ns : k * step;
        int q = ST ? k : dq;
#pragma unroll
        for (int t = 1; t < RAD; ++t, q += dq) {
          const cpx<R> w = tw[q];
          o[i][t] = DIR < 0 ? cmul(o[i][t], w) : cmulc(o[i][t], w);
        }
      }
      dft_radix<R, RAD, DIR>(o[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = tid + i * nthr;
    if (b < nb) {
      const int k = kk[i];
      int p = (b - k) * RAD + k;
#pragma unroll
      for (int t = 0; t < RAD; ++t, p += ns) buf[gpos(p) << lg] = o[i][t];
    }
  }
  __syncthreads();
}

// In-place transform of the line in buf (element p at buf[gpos(p) << lg]); every
// thread of the workgroup calls it after a barrier that follows the writes of the
// line.  ST: tw is the stage-layout table gen_stage_twiddles built.  The plan's
// radices are at most SMAX (a thread holds up to SMAX elements in a stage).
template <typename R, int DIR, bool ST, int SMAX>
__device__ void fft_gen(cpx<R>* buf, int lg, const GenPlan& gp, const cpx<R>* __restrict__ tw, int tid) {
  int ns = 1;
  const cpx<R>* t = tw;
  for (int s = 0; s < gp.nst; ++s) {
    const int r = gp.radix[s];
    switch (r) {
      case 2: gen_stage<R, 2, DIR, ST, SMAX>(buf, lg, gp.n, ns, t, tid, gp.nthr); break;
      case 3: gen_stage<R, 3, DIR, ST, SMAX>(buf, lg, gp.n, ns, t, tid, gp.nthr); break;
      case 4: gen_stage<R, 4, DIR, ST, SMAX>(buf, lg, gp.n, ns, t, tid, gp.nthr); break;
      case 5: gen_stage<R, 5, DIR, ST, SMAX>(buf, lg, gp.n, ns, t, tid, gp.nthr); break;
      case 6: if constexpr (SMAX >= 6) gen_stage<R, 6, DIR, ST, SMAX>(buf, lg, gp.n, ns, t, tid, gp.nthr); break;
      case 8: if constexpr (SMAX >= 8) gen_stage<R, 8, DIR, ST, SMAX>(buf, lg, gp.n, ns, t, tid, gp.nthr); break;
      case 9: if constexpr (SMAX >= 9) gen_stage<R, 9, DIR, ST, SMAX>(buf, lg, gp.n, ns, t, tid, gp.nthr); break;
      case 10: if constexpr (SMAX >= 10) gen_stage<R, 10, DIR, ST, SMAX>(buf, lg, gp.n, ns, t, tid, gp.nthr); break;
      case 12: if constexpr (SMAX >= 12) gen_stage<R, 12, DIR, ST, SMAX>(buf, lg, gp.n, ns, t, tid, gp.nthr); break;
      case 15: if constexpr (SMAX >= 15) gen_stage<R, 15, DIR, ST, SMAX>(buf, lg, gp.n, ns, t, tid, gp.nthr); break;
      default: if constexpr (SMAX >= 16) gen_stage<R, 16, DIR, ST, SMAX>(buf, lg, gp.n, ns, t, tid, gp.nthr); break;
    }
    if (ST && ns > 1) t += (size_t)ns * (r - 1);
    ns *= r;
  }
}

// The stage-layout twiddle table of plan gp (n - radix[0] entries) gathered into
// stw from the line's table tw by all nthr threads of the workgroup; the caller
// puts a barrier between this and the first use.
template <typename R>
__device__ void gen_stage_twiddles(cpx<R>* stw, const GenPlan& gp, const cpx<R>* __restrict__ tw, int tid,
                                   int nthr) {
  int ns = gp.radix[0], off = 0;
  for (int s = 1; s < gp.nst; ++s) {
    const int r = gp.radix[s], cnt = ns * (r - 1), step = gp.n / (ns * r);
    for (int q = tid; q < cnt; q += nthr) {
      const int t = q / ns + 1, k = q - (t - 1) * ns;
      stw[off + q] = tw[k * t * step];
    }
    off += cnt;
    ns *= r;
  }
}

// Pass A: forward transform of rows of length gp.n (stage radices up to SM).
template <typename R, typename TI, int SM>
__device__ __forceinline__ void rows_fwd_gen_body(const cpx<TI>* __restrict__ in, cpx<R>* __restrict__ out,
                                                  size_t in_rs, size_t out_rs, const GenPlan& gp,
                                                  const cpx<R>* __restrict__ tw, const int* __restrict__ skip) {
  extern __shared__ char dyn_lds[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(dyn_lds);
  const int rhs = blockIdx.y;
  if (skip != nullptr && skip[rhs] != 0) return;
  const int n = gp.n, tid = threadIdx.x;
  const size_t row = blockIdx.x;
  const cpx<TI>* src = in + (size_t)rhs * in_rs + row * n;
  {   // the row's loads issued together, then written to LDS
    cpx<R> x[kGenRowE];
#pragma unroll
    for (int i = 0; i < kGenRowE; ++i) {
      const int p = tid + i * gp.nthr;
      x[i] = p < n ? cvt<R>(src[p]) : cpx<R>{0, 0};
    }
#pragma unroll
    for (int i = 0; i < kGenRowE; ++i) {
      const int p = tid + i * gp.nthr;
      if (p < n) buf[gpos(p)] = x[i];
    }
  }
  __syncthreads();
  fft_gen<R, -1, false, SM>(buf, 0, gp, tw, tid);
  cpx<R>* dst = out + (size_t)rhs * out_rs + row * n;
  for (int i = tid; i < n; i += gp.nthr) dst[i] = buf[gpos(i)];
}
// stage radices up to 16, two waves per SIMD (up to 256 VGPRs)
template <typename R, typename TI>
__global__ __launch_bounds__(512) void k_rows_fwd_gen(const cpx<TI>* __restrict__ in, cpx<R>* __restrict__ out,
                                                       size_t in_rs, size_t out_rs, GenPlan gp,
                                                       const cpx<R>* __restrict__ tw, const int* __restrict__ skip) {
  rows_fwd_gen_body<R, TI, kGenStageMax>(in, out, in_rs, out_rs, gp, tw, skip);
}
// stage radices up to 12 at three waves per SIMD (168 VGPRs): three workgroups of
// four wavefronts share a CU
template <typename R, typename TI>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3))) void k_rows_fwd_gen3(
    const cpx<TI>* __restrict__ in, cpx<R>* __restrict__ out, size_t in_rs, size_t out_rs, GenPlan gp,
    const cpx<R>* __restrict__ tw, const int* __restrict__ skip) {
  rows_fwd_gen_body<R, TI, kGenRowSmaxLo>(in, out, in_rs, out_rs, gp, tw, skip);
}

// Strided axis, gp.tc adjacent columns per workgroup (their lines interleaved
// in LDS: element p of column g at gpos(p)*tc + g, so that loads and stores of a
// wavefront touch tc consecutive columns): element (o, p, c) at o*n*S + p*S + c.
// MODE 0: plain transform (slabs that no point of node field `fld` uses are skipped);
// MODE 1: forward transform, then for every node symbol multiply and inverse
// transform, storing the axis-0 indices whose rows use the node (need[n][p]).
template <typename R, int DIR, int MODE>
__global__ __launch_bounds__(gen_maxthr<R>()) void k_cols_gen(const cpx<R>* __restrict__ in, cpx<R>* __restrict__ out, int S,
                                                   int nfields, size_t in_rs, size_t out_rs, size_t in_fs,
                                                   size_t out_fs, GenPlan gp, const cpx<R>* __restrict__ tw,
                                                   const int* __restrict__ skip, const double* __restrict__ lam_ax,
                                                   const double* __restrict__ lam_in,
                                                   const NodeConst* __restrict__ nodes, int K, double scale,
                                                   const uint8_t* __restrict__ need,
                                                   const uint16_t* __restrict__ smask) {
  constexpr int E = gen_e<R>();
  constexpr bool ST = HP_GEN_LDS_TW != 0;
  extern __shared__ char dyn_lds[];
  const int z = blockIdx.z;
  const int rhs = (MODE == 0) ? z / nfields : z;
  const int fld = (MODE == 0) ? z % nfields : 0;
  if (skip != nullptr && skip[rhs] != 0) return;
  if (MODE == 0 && need != nullptr && need[(size_t)fld * gridDim.y + blockIdx.y] == 0) return;
  const int n = gp.n, tc = gp.tc, nthr = gp.nthr;
  const int lg = __builtin_ctz(tc);   // tc is a power of two
  const int g = threadIdx.x & (tc - 1), tl = threadIdx.x >> lg;
  int tile = blockIdx.x;
  if ((gridDim.x & 7) == 0) tile = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);   // XCD-aware
  const int c = tile * tc + g;
  const bool act = c < S;
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(dyn_lds) + g;
  const size_t obase = (size_t)blockIdx.y * n * S + (act ? c : 0);
  const cpx<R>* src = in + (size_t)rhs * in_rs + (size_t)fld * in_fs + obase;
  {   // the column's loads issued together, then written to LDS
    cpx<R> x[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int p = tl + i * nthr;
      x[i] = (act && p < n) ? src[(size_t)p * S] : cpx<R>{0, 0};
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int p = tl + i * nthr;
      if (p < n) buf[gpos(p) << lg] = x[i];
    }
  }
  if constexpr (ST) {   // the stage twiddle tables after the tc lines
    cpx<R>* stw = reinterpret_cast<cpx<R>*>(dyn_lds) + gen_line_slots(n) * tc;
    gen_stage_twiddles<R>(stw, gp, tw, threadIdx.x, nthr * tc);
    tw = stw;
  }
  __syncthreads();
  if constexpr (MODE == 0) {
    fft_gen<R, DIR, ST, gen_smax<R>(kGenCols)>(buf, lg, gp, tw, tl);
    if (act) {
      cpx<R>* dst = out + (size_t)rhs * out_rs + (size_t)fld * out_fs + obase;
      for (int p = tl; p < n; p += nthr) dst[(size_t)p * S] = buf[gpos(p) << lg];
    }
  } else {
    fft_gen<R, -1, ST, gen_smax<R>(kGenSym)>(buf, lg, gp, tw, tl);
    // the spectrum and lambda of this thread's elements p = tl + nthr * i
    cpx<R> vh[E];
    double lam[E];
    const double lc = act ? lam_in[c] : 0.0;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int p = tl + i * nthr;
      vh[i] = p < n ? buf[gpos(p) << lg] : cpx<R>{0, 0};
      lam[i] = p < n ? lam_ax[p] + lc : 0.0;
    }
    cpx<R>* dst = out + (size_t)rhs * out_rs + obase;
    for (int nd = 0; nd < K; ++nd) {
      const NodeConst nc = nodes[nd];
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int p = tl + i * nthr;
        if (p < n) {
          const double dre = nc.are - nc.gre * lam[i];
          const double dim = nc.aim - nc.gim * lam[i];
          cpx<R> q;
          if constexpr (sizeof(R) == 8) {
            const double inv = scale * recip(dre * dre + dim * dim);
            q = {dre * inv, -dim * inv};
          } else {
            const float fr = (float)dre, fi = (float)dim;
            const float inv = (float)scale * recip(fr * fr + fi * fi);
            q = {fr * inv, -fi * inv};
          }
          buf[gpos(p) << lg] = cmul(vh[i], q);
        }
      }
      __syncthreads();
      fft_gen<R, +1, ST, gen_smax<R>(kGenSym)>(buf, lg, gp, tw, tl);
      if (act) {
        if (smask != nullptr) {   // one packed word per thread and node: bit i = element tl + i nthr
          const unsigned m = smask[(size_t)nd * nthr + tl];
          for (int i = 0; i < E; ++i)
            if ((m >> i) & 1u) {
              const int p = tl + i * nthr;
              dst[(size_t)nd * out_fs + (size_t)p * S] = buf[gpos(p) << lg];
            }
        } else {
          const uint8_t* nn = need + (size_t)nd * n;
          for (int p = tl; p < n; p += nthr)
            if (nn[p]) dst[(size_t)nd * out_fs + (size_t)p * S] = buf[gpos(p) << lg];
        }
      }
    }
  }
}

// Pass C: inverse transform along rows of every node the row uses, and the
// hat-weighted combine (weights 1-t on node A, t on node B of each point).
template <typename R, typename TO, bool ACC, int IM>
__global__ __launch_bounds__(gen_maxthr<R>()) void k_rows_combine_gen(const cpx<R>* __restrict__ fields, size_t fs,
                                                           size_t frs, const double* __restrict__ pos,
                                                           const uint64_t* __restrict__ rowmask,
                                                           cpx<TO>* __restrict__ out, size_t out_rs, int K, int M,
                                                           int Mt, int mo, GenPlan gp,
                                                           const cpx<R>* __restrict__ tw,
                                                           const int* __restrict__ skip, int ord,
                                                           const double* __restrict__ lag,
                                                           const double* __restrict__ posa, int Ma) {
  constexpr bool LAG = IM == kInterpLagrange;
  extern __shared__ char dyn_lds[];
  cpx<R>* buf = reinterpret_cast<cpx<R>*>(dyn_lds);
  __shared__ double slag[LAG ? kLagTable : 1];
  const int rhs = blockIdx.y;
  if (skip != nullptr && skip[rhs] != 0) return;
  const int n = gp.n, tid = threadIdx.x, nthr = gp.nthr;
  if constexpr (LAG) {
    for (int i = tid; i < kLagTable; i += nthr) slag[i] = lag[i];
    __syncthreads();
  }
  const size_t row = blockIdx.x, rbase = row * n;
  int ab[gen_e<R>()];
  R tt[gen_e<R>()], uu[gen_e<R>()];
  cpx<R> acc[gen_e<R>()];
#pragma unroll
  for (int i = 0; i < gen_e<R>(); ++i) {
    const int p = tid + i * nthr;
    ab[i] = 0xffff;
    tt[i] = (R)0;
    uu[i] = (R)0;
    if (p < n)
      interp_record<R, IM>(pos[rbase + p], IM == kInterpBilinear ? posa[rbase + p] : 0.0, M, Mt, mo, Ma, ord, slag,
                           ab[i], tt[i], uu[i]);
    acc[i] = {0, 0};
  }
  const uint64_t rm = rowmask[row];
  const cpx<R>* fr = fields + (size_t)rhs * frs + rbase;
  constexpr bool ST = HP_GEN_LDS_TW != 0;
  if constexpr (ST) {   // the stage twiddle tables after the line
    cpx<R>* stw = buf + gen_line_slots(n);
    gen_stage_twiddles<R>(stw, gp, tw, tid, nthr);
    tw = stw;
  }
  for (int nd = 0; nd < K; ++nd) {
    if (((rm >> nd) & 1ull) == 0) continue;
    {   // the node row's loads issued together, then written to LDS
      cpx<R> x[gen_e<R>()];
#pragma unroll
      for (int i = 0; i < gen_e<R>(); ++i) {
        const int p = tid + i * nthr;
        x[i] = p < n ? fr[(size_t)nd * fs + p] : cpx<R>{0, 0};
      }
#pragma unroll
      for (int i = 0; i < gen_e<R>(); ++i) {
        const int p = tid + i * nthr;
        if (p < n) buf[gpos(p)] = x[i];
      }
    }
    __syncthreads();
    fft_gen<R, +1, ST, gen_smax<R>(kGenComb)>(buf, 0, gp, tw, tid);
#pragma unroll
    for (int i = 0; i < gen_e<R>(); ++i) {
      const int p = tid + i * nthr;
      if (p < n) {
        const R w = interp_weight<R, IM>(ab[i], tt[i], uu[i], nd, ord, slag);
        const cpx<R> x = buf[gpos(p)];
        acc[i].re += w * x.re;
        acc[i].im += w * x.im;
      }
    }
  }
  cpx<TO>* dst = out + (size_t)rhs * out_rs + rbase;
#pragma unroll
  for (int i = 0; i < gen_e<R>(); ++i) {
    const int p = tid + i * nthr;
    if (p < n) {
      if constexpr (ACC) {
        const cpx<TO> o = dst[p];
        dst[p] = {o.re + (TO)acc[i].re, o.im + (TO)acc[i].im};
      } else {
        dst[p] = cvt<TO>(acc[i]);
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
                          const void* tw, const int* skip, hipStream_t st, const hipEvent_t* tev) {
      using C = RowCfg<R, N>;
      dim3 grid((rows + C::G - 1) / C::G, nrhs);
      HP_PASS_LAUNCH(tev, (k_rows_fwd<R, TI, N>), grid, dim3(C::THREADS), 0, st, (const cpx<TI>*)in,
                     (cpx<R>*)out, rows, in_rs, out_rs, (const cpx<R>*)tw, skip);
      return hipGetLastError();
    }
  };
};

// ---- mixed-radix launch helpers
bool make_gen_plan(int n, int E, int maxthr, GenPlan* gp, int order, int nthr_req, int smax) {
  static const int kRadices[] = {16, 15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
  static const int kPrimeOrder[4] = {4, 2, 3, 5};
  if (n < 2 || n > kGenMaxN || order < 0 || order >= kGenOrders) return false;
  GenPlan g{};
  g.n = n;
  g.tc = 1;
  g.smax = smax;
  int m = n;
  if (order == 3) {   // radices 4, 2, 3, 5 only, each as often as it divides what is left
    for (int r : kPrimeOrder)
      while (m % r == 0 && g.nst < kGenMaxStages) { g.radix[g.nst++] = r; m /= r; }
  } else {            // the largest radix that divides what is left, first
    while (m > 1 && g.nst < kGenMaxStages) {
      int pick = 0;
      for (int r : kRadices)
        if (r <= smax && m % r == 0) { pick = r; break; }
      if (pick == 0) break;
      g.radix[g.nst++] = pick;
      m /= pick;
    }
    if (order == 1) {                       // ascending
      for (int i = 0, j = g.nst - 1; i < j; ++i, --j) { const int x = g.radix[i]; g.radix[i] = g.radix[j]; g.radix[j] = x; }
    } else if (order == 2 && g.nst > 1) {   // the largest stage last
      const int x = g.radix[0];
      for (int i = 0; i + 1 < g.nst; ++i) g.radix[i] = g.radix[i + 1];
      g.radix[g.nst - 1] = x;
    }
  }
  if (m != 1) return false;
  auto fits = [&](int t) {
    bool ok = (size_t)t * E >= (size_t)n;
    for (int s = 0; s < g.nst && ok; ++s) {
      const int r = g.radix[s];
      ok = (n / r + t - 1) / t <= smax / r;
    }
    return ok;
  };
  if (nthr_req > 0) {
    if (nthr_req % 64 != 0 || nthr_req > maxthr || !fits(nthr_req)) return false;
    g.nthr = nthr_req;
    *gp = g;
    return true;
  }
  // the smallest power of two of wavefronts that fits: workgroups of 1, 2, 4 or 8
  // wavefronts fill a CU's wave slots evenly at two waves per SIMD (5-7 would leave
  // slots empty beside a second workgroup that does not fit)
  for (int t = 64; t <= maxthr; t *= 2)
    if (fits(t)) { g.nthr = t; *gp = g; return true; }
  for (int t = 64; t <= maxthr; t += 64)
    if (fits(t)) { g.nthr = t; *gp = g; return true; }
  return false;
}

// A pass's plan with its run-time choices, or the built-in one when they do not fit.
static bool tuned_gen_plan(int n, int E, int maxthr, const PassTune& t, GenPlan* gp, int smax) {
  if ((t.nthr > 0 || t.order > 0) && make_gen_plan(n, E, maxthr, gp, t.order, t.nthr, smax)) return true;
  return make_gen_plan(n, E, maxthr, gp, 0, 0, smax);
}

// Pass A's stage-radix cap for a mixed-radix row length (either precision): 12 (the
// kernel at three waves per SIMD) unless that plan needs more threads than 256 and than
// the plan at 16 does (the 5 of 2880 = 2^6 3^2 5 needs radix 10 and 288 threads under 12).
int gen_rows_smax(int real_kind, int n) {
  (void)real_kind;
  GenPlan lo, hi;
  const bool okl = make_gen_plan(n, kGenRowE, 512, &lo, 0, 0, kGenRowSmaxLo);
  const bool okh = make_gen_plan(n, kGenRowE, 512, &hi, 0, 0, kGenStageMax);
  if (okl && (!okh || lo.nthr <= 256 || lo.nthr <= hi.nthr)) return kGenRowSmaxLo;
  return okh ? kGenStageMax : kGenRowSmaxLo;
}

bool gen_length_ok(int n) {
  bool ok = true;
  for (int k = kGenRows; k <= kGenComb && ok; ++k) {
    GenPlan a;
    const int e64 = k == kGenRows ? kGenRowE : gen_e<double>(), e32 = k == kGenRows ? kGenRowE : gen_e<float>();
    const int t64 = k == kGenRows ? 512 : gen_maxthr<double>(), t32 = k == kGenRows ? 512 : gen_maxthr<float>();
    const int s64 = k == kGenRows ? gen_rows_smax(0, n) : gen_smax<double>(k);
    const int s32 = k == kGenRows ? gen_rows_smax(1, n) : gen_smax<float>(k);
    ok = make_gen_plan(n, e64, t64, &a, 0, 0, s64) && make_gen_plan(n, e32, t32, &a, 0, 0, s32);
  }
  return ok;
}

// Column passes: a power of two of adjacent columns per workgroup (at most 8) within
// the thread limit and up to 144 KiB of LDS.
template <typename R>
static bool col_tc_fits(int n, int S, int nthr, int tc) {
  return tc >= 1 && tc <= 8 && (tc & (tc - 1)) == 0 && tc * nthr <= gen_maxthr<R>() &&
         (gen_line_slots(n) * tc + (HP_GEN_LDS_TW ? n : 0)) * sizeof(cpx<R>) <= (size_t)144 * 1024 && tc <= S;
}

template <typename R>
static bool make_col_plan(int n, int S, int mode, GenPlan* gp, const PassTune& t = PassTune{}) {
  if (!tuned_gen_plan(n, gen_e<R>(), gen_maxthr<R>(), t, gp, gen_smax<R>(mode == 1 ? kGenSym : kGenCols))) return false;
  if (t.tc > 0 && col_tc_fits<R>(n, S, gp->nthr, t.tc)) {
    gp->tc = t.tc;
    return true;
  }
  // up to 256 threads per workgroup, so that two or more workgroups share a CU and
  // one's barriers overlap another's work
  int tc = 1;
  while (tc < 8 && tc * 2 * gp->nthr <= 256 && col_tc_fits<R>(n, S, gp->nthr, tc * 2)) tc *= 2;
  gp->tc = tc;
  return true;
}

bool combine_splits_ok(int real_kind, int n);   // pass C of this length can split its nodes

bool cols_use_gen(int real_kind, int n) { return !is_pow2_len(n) || (real_kind == 0 && n > 2048); }


int tune_candidates(int real_kind, int kind, int n, int S, int mode, int K, PassTune* out, int max) {
  int cnt = 0;
  auto push = [&](const PassTune& t) {
    if (cnt < max) out[cnt++] = t;
  };
  if (kind == kTuneCols ? !cols_use_gen(real_kind, n) : is_pow2_len(n)) {
    // compile-time tiles; the node groups of the symbol pass and the node splits
    // of pass C vary
    if (kind == kTuneCols && mode == 1)
      for (int ng = 1; ng <= K && ng <= kMaxNodes; ng *= 2) push(PassTune{0, 0, 0, ng});
    if (kind == kTuneCombine && combine_splits_ok(real_kind, n)) {
      push(PassTune{0, 0, 0, 1});
      push(PassTune{0, 0, 0, kCombineSplits});
    }
    return cnt;
  }
  const int E = kind == kTuneRows ? kGenRowE : (real_kind == 0 ? gen_e<double>() : gen_e<float>());
  const int maxthr = kind == kTuneRows ? 512 : (real_kind == 0 ? gen_maxthr<double>() : gen_maxthr<float>());
  const int gk = kind == kTuneRows ? kGenRows : kind == kTuneCols ? (mode == 1 ? kGenSym : kGenCols) : kGenComb;
  const int smax = kind == kTuneRows ? gen_rows_smax(real_kind, n)
                                     : (real_kind == 0 ? gen_smax<double>(gk) : gen_smax<float>(gk));
  for (int order = 0; order < kGenOrders; ++order) {
    GenPlan g;
    if (!make_gen_plan(n, E, maxthr, &g, order, 0, smax)) continue;
    // the smallest thread count that fits and up to three larger ones, and the
    // built-in (power-of-two) one
    int tmin = 0;
    for (int t = 64; t <= maxthr && tmin == 0; t += 64) {
      GenPlan h;
      if (make_gen_plan(n, E, maxthr, &h, order, t, smax)) tmin = t;
    }
    int cand[5], nc = 0;
    for (int t = tmin, k = 0; tmin > 0 && t <= maxthr && k < 4; t += 64, ++k) cand[nc++] = t;
    if (g.nthr >= tmin + 4 * 64) cand[nc++] = g.nthr;
    for (int ci = 0; ci < nc; ++ci) {
      const int t = cand[ci];
      GenPlan h;
      if (!make_gen_plan(n, E, maxthr, &h, order, t, smax)) continue;
      if (kind != kTuneCols) {
        push(PassTune{t, 0, order, 0});
        continue;
      }
      for (int tc = 1; tc <= 8; tc *= 2) {
        const bool ok = real_kind == 0 ? col_tc_fits<double>(n, S, t, tc) : col_tc_fits<float>(n, S, t, tc);
        if (ok) push(PassTune{t, tc, order, 0});
      }
    }
  }
  return cnt;
}

template <typename K>
static void allow_dynamic_lds(K kernel, size_t bytes) {
  // lines longer than 64 KiB of LDS need the limit raised once per kernel
  if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename R, typename TI>
static hipError_t rows_fwd_gen(const GenPlan& gp, const void* in, void* out, int rows, size_t in_rs, size_t out_rs,
                               int nrhs, const void* tw, const int* skip, hipStream_t st, const hipEvent_t* tev) {
  const size_t lds = gen_line_slots(gp.n) * sizeof(cpx<R>);
  if (gp.smax <= kGenRowSmaxLo) {
    allow_dynamic_lds(k_rows_fwd_gen3<R, TI>, lds);
    HP_PASS_LAUNCH(tev, (k_rows_fwd_gen3<R, TI>), dim3(rows, nrhs), dim3(gp.nthr), lds, st, (const cpx<TI>*)in,
                   (cpx<R>*)out, in_rs, out_rs, gp, (const cpx<R>*)tw, skip);
  } else {
    allow_dynamic_lds(k_rows_fwd_gen<R, TI>, lds);
    HP_PASS_LAUNCH(tev, (k_rows_fwd_gen<R, TI>), dim3(rows, nrhs), dim3(gp.nthr), lds, st, (const cpx<TI>*)in,
                   (cpx<R>*)out, in_rs, out_rs, gp, (const cpx<R>*)tw, skip);
  }
  return hipGetLastError();
}

template <typename R>
static hipError_t cols_gen(const GenPlan& gp, const ColsArgs& a, hipStream_t st) {
  const size_t lds = (gen_line_slots(gp.n) * gp.tc + (HP_GEN_LDS_TW ? gp.n : 0)) * sizeof(cpx<R>);
  dim3 grid((a.S + gp.tc - 1) / gp.tc, a.outer, a.mode == 0 ? a.nrhs * a.nfields : a.nrhs);
  const cpx<R>* in = (const cpx<R>*)a.in;
  cpx<R>* out = (cpx<R>*)a.out;
  const cpx<R>* tw = (const cpx<R>*)a.tw;
  if (a.mode == 1) {
    allow_dynamic_lds(k_cols_gen<R, -1, 1>, lds);
    const uint16_t* sm = (a.store_mask_thr == gp.nthr && a.store_mask_thr > 0) ? a.store_mask : nullptr;
    HP_PASS_LAUNCH(a.tev, (k_cols_gen<R, -1, 1>), grid, dim3(gp.nthr * gp.tc), lds, st, in, out, a.S, a.nfields, a.in_rs,
                       a.out_rs, a.in_fs, a.out_fs, gp, tw, a.skip, a.lam_ax, a.lam_in, a.nodes, a.K, a.scale,
                       a.store_need, sm);
  } else if (a.dir < 0) {
    allow_dynamic_lds(k_cols_gen<R, -1, 0>, lds);
    HP_PASS_LAUNCH(a.tev, (k_cols_gen<R, -1, 0>), grid, dim3(gp.nthr * gp.tc), lds, st, in, out, a.S, a.nfields, a.in_rs,
                       a.out_rs, a.in_fs, a.out_fs, gp, tw, a.skip, a.lam_ax, a.lam_in, a.nodes, a.K, a.scale,
                       a.slab_need, nullptr);
  } else {
    allow_dynamic_lds(k_cols_gen<R, +1, 0>, lds);
    HP_PASS_LAUNCH(a.tev, (k_cols_gen<R, +1, 0>), grid, dim3(gp.nthr * gp.tc), lds, st, in, out, a.S, a.nfields, a.in_rs,
                       a.out_rs, a.in_fs, a.out_fs, gp, tw, a.skip, a.lam_ax, a.lam_in, a.nodes, a.K, a.scale,
                       a.slab_need, nullptr);
  }
  return hipGetLastError();
}

template <typename R, typename TO, bool ACC, int IM>
static hipError_t combine_gen_l(const GenPlan& gp, const CombineArgs& a, hipStream_t st) {
  const size_t lds = (gen_line_slots(gp.n) + (HP_GEN_LDS_TW ? gp.n : 0)) * sizeof(cpx<R>);
  allow_dynamic_lds(k_rows_combine_gen<R, TO, ACC, IM>, lds);
  HP_PASS_LAUNCH(a.tev, (k_rows_combine_gen<R, TO, ACC, IM>), dim3(a.rows, a.nrhs), dim3(gp.nthr), lds, st,
                     (const cpx<R>*)a.fields, a.fs, a.frs, a.pos, a.rowmask, (cpx<TO>*)a.out, a.out_rs, a.K, a.M,
                     a.Mt, a.mo, gp, (const cpx<R>*)a.tw, a.skip, a.order, a.lag, a.posa, a.Ma);
  return hipGetLastError();
}
static int interp_mode(const CombineArgs& a) {
  return a.order >= 2 ? kInterpLagrange : (a.Ma >= 2 ? kInterpBilinear : kInterpLinear);
}
template <typename R, typename TO, bool ACC>
static hipError_t combine_gen(const GenPlan& gp, const CombineArgs& a, hipStream_t st) {
  switch (interp_mode(a)) {
    case kInterpLagrange: return combine_gen_l<R, TO, ACC, kInterpLagrange>(gp, a, st);
    case kInterpBilinear: return combine_gen_l<R, TO, ACC, kInterpBilinear>(gp, a, st);
    default: return combine_gen_l<R, TO, ACC, kInterpLinear>(gp, a, st);
  }
}

hipError_t launch_rows_fwd(int real_kind, int in_kind, int n, const void* in, void* out, int rows,
                           size_t in_rs, size_t out_rs, int nrhs, const void* tw, const int* skip,
                           const PassTune& tune, hipStream_t st, const hipEvent_t* tev) {
  if (!is_pow2_len(n)) {
    GenPlan gp;
    if (!tuned_gen_plan(n, kGenRowE, 512, tune, &gp, gen_rows_smax(real_kind, n))) return hipErrorInvalidValue;
    if (real_kind == 0) {
      if (in_kind != 0) return hipErrorInvalidValue;
      return rows_fwd_gen<double, double>(gp, in, out, rows, in_rs, out_rs, nrhs, tw, skip, st, tev);
    }
    if (in_kind == 0) return rows_fwd_gen<float, double>(gp, in, out, rows, in_rs, out_rs, nrhs, tw, skip, st, tev);
    return rows_fwd_gen<float, float>(gp, in, out, rows, in_rs, out_rs, nrhs, tw, skip, st, tev);
  }
  if (real_kind == 0) {
    if (in_kind != 0) return hipErrorInvalidValue;
    return dispatch_n<RowsFwdL<double, double>::F>(n, in, out, rows, in_rs, out_rs, nrhs, tw, skip, st, tev);
  }
  if (in_kind == 0)
    return dispatch_n<RowsFwdL<float, double>::F>(n, in, out, rows, in_rs, out_rs, nrhs, tw, skip, st, tev);
  return dispatch_n<RowsFwdL<float, float>::F>(n, in, out, rows, in_rs, out_rs, nrhs, tw, skip, st, tev);
}

template <typename R>
struct ColsL {
  template <int N>
  struct F {
    static hipError_t run(const ColsArgs& a, hipStream_t st) {
      using C0 = ColsCfg<R, N, 0>;
      using C1 = ColsCfg<R, N, 1>;
      if constexpr (sizeof(R) == 8 && N > 2048) {
        return hipErrorInvalidValue;   // the FP64 column tile would not fit in LDS
      } else {
        const int TC = a.mode == 1 ? C1::TC : C0::TC;
        const int tiles = (a.S + TC - 1) / TC;
        // symbol pass: node groups so that at least ~512 workgroups run (small grids),
        // or the tuned count
        const int ng = a.mode != 1 ? 1
                       : a.tune.ng > 0 ? std::min(a.K, a.tune.ng)
                                       : std::max(1, std::min(a.K, (512 + tiles - 1) / tiles));
        dim3 grid(tiles, a.mode == 1 ? ng : a.outer, a.mode == 0 ? a.nrhs * a.nfields : a.nrhs);
        const cpx<R>* in = (const cpx<R>*)a.in;
        cpx<R>* out = (cpx<R>*)a.out;
        const cpx<R>* tw = (const cpx<R>*)a.tw;
        if (a.mode == 1)
          HP_PASS_LAUNCH(a.tev, (k_cols<R, R, N, -1, 1>), grid, dim3(C1::THREADS), 0, st, in, out, a.S,
                             a.nfields, a.in_rs, a.out_rs, a.in_fs, a.out_fs, tw, a.skip, a.lam_ax,
                             a.lam_in, a.nodes, a.K, a.scale, a.store_mask, a.slab_need);
        else if (a.dir < 0)
          HP_PASS_LAUNCH(a.tev, (k_cols<R, R, N, -1, 0>), grid, dim3(C0::THREADS), 0, st, in, out, a.S,
                             a.nfields, a.in_rs, a.out_rs, a.in_fs, a.out_fs, tw, a.skip, a.lam_ax,
                             a.lam_in, a.nodes, a.K, a.scale, a.store_mask, a.slab_need);
        else
          HP_PASS_LAUNCH(a.tev, (k_cols<R, R, N, +1, 0>), grid, dim3(C0::THREADS), 0, st, in, out, a.S,
                             a.nfields, a.in_rs, a.out_rs, a.in_fs, a.out_fs, tw, a.skip, a.lam_ax,
                             a.lam_in, a.nodes, a.K, a.scale, a.store_mask, a.slab_need);
        return hipGetLastError();
      }
    }
  };
};

hipError_t launch_cols(const ColsArgs& a, hipStream_t st) {
  if (cols_use_gen(a.real_kind, a.n)) {
    GenPlan gp;
    if (a.real_kind == 0)
      return make_col_plan<double>(a.n, a.S, a.mode, &gp, a.tune) ? cols_gen<double>(gp, a, st) : hipErrorInvalidValue;
    return make_col_plan<float>(a.n, a.S, a.mode, &gp, a.tune) ? cols_gen<float>(gp, a, st) : hipErrorInvalidValue;
  }
  if (a.real_kind == 0) return dispatch_n<ColsL<double>::F>(a.n, a, st);
  return dispatch_n<ColsL<float>::F>(a.n, a, st);
}

template <typename R, typename TO, int N, bool ACC, int NS>
static void combine_launch(const CombineArgs& a, dim3 grid, hipStream_t st) {
  using C = CombCfg<R, N>;
  const dim3 block(C::THREADS * NS);
  switch (interp_mode(a)) {
    case kInterpLagrange:
      HP_PASS_LAUNCH(a.tev, (k_rows_combine<R, TO, N, ACC, kInterpLagrange, NS>), grid, block, 0, st,
                         (const cpx<R>*)a.fields, a.fs, a.frs, a.pos, a.grpmask, a.rowmask, (cpx<TO>*)a.out,
                         a.out_rs, a.rows, a.K, a.M, a.Mt, a.mo, (const cpx<R>*)a.tw, a.skip, a.order, a.lag, a.posa,
                         a.Ma);
      break;
    case kInterpBilinear:
      HP_PASS_LAUNCH(a.tev, (k_rows_combine<R, TO, N, ACC, kInterpBilinear, NS>), grid, block, 0, st,
                         (const cpx<R>*)a.fields, a.fs, a.frs, a.pos, a.grpmask, a.rowmask, (cpx<TO>*)a.out,
                         a.out_rs, a.rows, a.K, a.M, a.Mt, a.mo, (const cpx<R>*)a.tw, a.skip, a.order, a.lag, a.posa,
                         a.Ma);
      break;
    default:
      HP_PASS_LAUNCH(a.tev, (k_rows_combine<R, TO, N, ACC, kInterpLinear, NS>), grid, block, 0, st,
                         (const cpx<R>*)a.fields, a.fs, a.frs, a.pos, a.grpmask, a.rowmask, (cpx<TO>*)a.out,
                         a.out_rs, a.rows, a.K, a.M, a.Mt, a.mo, (const cpx<R>*)a.tw, a.skip, a.order, a.lag, a.posa,
                         a.Ma);
  }
}

template <typename R, typename TO, bool ACC>
struct CombineL {
  template <int N>
  struct F {
    static hipError_t run(const CombineArgs& a, hipStream_t st) {
      using C = CombCfg<R, N>;
      if constexpr (wave_line_fits<R, N>() && (HP_WAVE_COMB & (sizeof(R) == 8 ? 2 : 1)) != 0) {
        const dim3 wgrid((a.rows + kWaveRows - 1) / kWaveRows, a.nrhs);
        switch (interp_mode(a)) {
          case kInterpLagrange:
            HP_PASS_LAUNCH(a.tev, (k_comb_wave<R, TO, N, ACC, kInterpLagrange>), wgrid, dim3(64 * kWaveRows), 0, st,
                           (const cpx<R>*)a.fields, a.fs, a.frs, a.pos, a.rowmask, (cpx<TO>*)a.out, a.out_rs,
                           a.rows, a.M, a.Mt, a.mo, (const cpx<R>*)a.tw, a.skip, a.order, a.lag, a.posa, a.Ma);
            break;
          case kInterpBilinear:
            HP_PASS_LAUNCH(a.tev, (k_comb_wave<R, TO, N, ACC, kInterpBilinear>), wgrid, dim3(64 * kWaveRows), 0, st,
                           (const cpx<R>*)a.fields, a.fs, a.frs, a.pos, a.rowmask, (cpx<TO>*)a.out, a.out_rs,
                           a.rows, a.M, a.Mt, a.mo, (const cpx<R>*)a.tw, a.skip, a.order, a.lag, a.posa, a.Ma);
            break;
          default:
            HP_PASS_LAUNCH(a.tev, (k_comb_wave<R, TO, N, ACC, kInterpLinear>), wgrid, dim3(64 * kWaveRows), 0, st,
                           (const cpx<R>*)a.fields, a.fs, a.frs, a.pos, a.rowmask, (cpx<TO>*)a.out, a.out_rs,
                           a.rows, a.M, a.Mt, a.mo, (const cpx<R>*)a.tw, a.skip, a.order, a.lag, a.posa, a.Ma);
        }
        return hipGetLastError();
      }
      dim3 grid((a.rows + C::G - 1) / C::G, a.nrhs);
      if constexpr (combine_splits_fit<R, N>()) {
        // node splits when the row groups alone would leave most of the chip idle, or
        // as tuned (the tuner's node-group field: 1 or kCombineSplits).  The choice
        // depends on the grid only, so that a batch sums in the order a single field does.
        const int groups = (int)grid.x;
        const int ns = a.tune.ng > 0 ? a.tune.ng : (groups < 512 ? kCombineSplits : 1);
        if (ns == kCombineSplits) {
          combine_launch<R, TO, N, ACC, kCombineSplits>(a, grid, st);
          return hipGetLastError();
        }
      }
      combine_launch<R, TO, N, ACC, 1>(a, grid, st);
      return hipGetLastError();
    }
  };
};

bool combine_splits_ok(int real_kind, int n) {
  switch (n) {
    case 128: return real_kind == 0 ? combine_splits_fit<double, 128>() : combine_splits_fit<float, 128>();
    case 256: return real_kind == 0 ? combine_splits_fit<double, 256>() : combine_splits_fit<float, 256>();
    case 512: return real_kind == 0 ? combine_splits_fit<double, 512>() : combine_splits_fit<float, 512>();
    case 1024: return real_kind == 0 ? combine_splits_fit<double, 1024>() : combine_splits_fit<float, 1024>();
    default: return false;
  }
}

hipError_t launch_combine(const CombineArgs& a, hipStream_t st) {
  if (!is_pow2_len(a.n)) {
    GenPlan gp;
    if (a.real_kind == 0
            ? !tuned_gen_plan(a.n, gen_e<double>(), gen_maxthr<double>(), a.tune, &gp, gen_smax<double>(kGenComb))
            : !tuned_gen_plan(a.n, gen_e<float>(), gen_maxthr<float>(), a.tune, &gp, gen_smax<float>(kGenComb)))
      return hipErrorInvalidValue;
    if (a.real_kind == 0) {
      if (a.out_kind != 0) return hipErrorInvalidValue;
      return a.accumulate ? combine_gen<double, double, true>(gp, a, st) : combine_gen<double, double, false>(gp, a, st);
    }
    if (a.out_kind == 0)
      return a.accumulate ? combine_gen<float, double, true>(gp, a, st) : combine_gen<float, double, false>(gp, a, st);
    if (a.accumulate) return hipErrorInvalidValue;
    return combine_gen<float, float, false>(gp, a, st);
  }
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
    case 8: return SymCfg<R, 8>::T;
    case 16: return SymCfg<R, 16>::T;
    case 32: return SymCfg<R, 32>::T;
    case 64: return SymCfg<R, 64>::T;
    case 128: return SymCfg<R, 128>::T;
    case 256: return SymCfg<R, 256>::T;
    case 512: return SymCfg<R, 512>::T;
    case 1024: return SymCfg<R, 1024>::T;
    case 2048: return SymCfg<R, 2048>::T;
    case 4096: return SymCfg<R, 4096>::T;
    default: return 1;
  }
}

int symbol_pass_line_threads(int real_kind, int n) {
  return real_kind == 0 ? sym_line_threads<double>(n) : sym_line_threads<float>(n);
}

int gen_symbol_line_threads(int real_kind, int n) {
  GenPlan g;
  const bool ok = real_kind == 0
                      ? make_gen_plan(n, gen_e<double>(), gen_maxthr<double>(), &g, 0, 0, gen_smax<double>(kGenSym))
                      : make_gen_plan(n, gen_e<float>(), gen_maxthr<float>(), &g, 0, 0, gen_smax<float>(kGenSym));
  return ok ? g.nthr : 0;
}
int gen_symbol_elems(int real_kind) { return real_kind == 0 ? gen_e<double>() : gen_e<float>(); }

int combine_group_rows(int real_kind, int n) {
  return real_kind == 0 ? group_rows<double>(n) : group_rows<float>(n);
}

// ---------------------------------------------------------------- stencil
// (P u)(x) = gamma^2 sum_j (u(x+e_j) + u(x-e_j)) / h_j^2 + beta u(x),
// beta = omega^2 + i omega a - 2 gamma^2 sum_j 1/h_j^2; periodic indices.
// coef holds {gamma^2, beta} per point.
// (P u)(x_i) for one point i of one field ur (periodic neighbours of any length);
// index arithmetic in 32 bits (every grid has fewer than 2^32 points): 64-bit
// division is a long software sequence on the GPU.
template <typename R, typename TI, int DIM>
__device__ __forceinline__ cpx<R> stencil_point(const cpx<TI>* __restrict__ ur, const cpx<R>* __restrict__ coef,
                                                size_t i, int n0, int n1, int n2, R ih0, R ih1, R ih2) {
  cpx<R> lap;
  auto nxt = [](int k, int n) { return k + 1 == n ? 0 : k + 1; };
  auto prv = [](int k, int n) { return k == 0 ? n - 1 : k - 1; };
  const uint32_t i32 = (uint32_t)i;
  if constexpr (DIM == 2) {
    const int i1 = (int)(i32 % (uint32_t)n1), i0 = (int)(i32 / (uint32_t)n1);
    const size_t r0 = (size_t)i0 * n1;
    const size_t up = (size_t)nxt(i0, n0) * n1, dn = (size_t)prv(i0, n0) * n1;
    const cpx<R> a = cvt<R>(ur[r0 + nxt(i1, n1)]), b = cvt<R>(ur[r0 + prv(i1, n1)]);
    const cpx<R> c = cvt<R>(ur[up + i1]), d = cvt<R>(ur[dn + i1]);
    lap = {(a.re + b.re) * ih1 + (c.re + d.re) * ih0, (a.im + b.im) * ih1 + (c.im + d.im) * ih0};
  } else {
    const uint32_t q2 = i32 / (uint32_t)n2;
    const int i2 = (int)(i32 - q2 * (uint32_t)n2);
    const int i1 = (int)(q2 % (uint32_t)n1);
    const int i0 = (int)(q2 / (uint32_t)n1);
    const size_t s1 = n2, s0 = (size_t)n1 * n2;
    const size_t b0 = (size_t)i0 * s0, b1 = (size_t)i1 * s1;
    const cpx<R> a = cvt<R>(ur[b0 + b1 + nxt(i2, n2)]), b = cvt<R>(ur[b0 + b1 + prv(i2, n2)]);
    const cpx<R> c = cvt<R>(ur[b0 + (size_t)nxt(i1, n1) * s1 + i2]);
    const cpx<R> d = cvt<R>(ur[b0 + (size_t)prv(i1, n1) * s1 + i2]);
    const cpx<R> e = cvt<R>(ur[(size_t)nxt(i0, n0) * s0 + b1 + i2]);
    const cpx<R> q = cvt<R>(ur[(size_t)prv(i0, n0) * s0 + b1 + i2]);
    lap = {(a.re + b.re) * ih2 + (c.re + d.re) * ih1 + (e.re + q.re) * ih0,
           (a.im + b.im) * ih2 + (c.im + d.im) * ih1 + (e.im + q.im) * ih0};
  }
  const cpx<R> g2 = coef[2 * i], be = coef[2 * i + 1];
  const cpx<R> uc = cvt<R>(ur[i]);
  return cadd(cmul(g2, lap), cmul(be, uc));
}

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
  const cpx<R> r = stencil_point<R, TI, DIM>(u + (size_t)rhs * u_rs, coef, i, n0, n1, n2, ih0, ih1, ih2);
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
    dst[(size_t)threadIdx.x * kRedBlocks] = {re, im};   // partials are stored [slot][block]
  }
  __syncthreads();
}

__device__ __forceinline__ double cabs2(cpx<double> a) { return a.re * a.re + a.im * a.im; }

// Workgroup barrier that orders LDS only: global stores issued before it (the
// solver state) are not waited for, since no thread of the block reads them back.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum the kRedBlocks block partials of `cnt` slots of right-hand side `rhs`
// into sums[] in a fixed order (wave w handles slots w, w + nw, ...; kSlotsPerWave
// slots per round, so that each lane has 16 partial loads of a round in flight
// before the first add).
static_assert(kRedBlocks % 64 == 0, "partials per slot must fill whole wavefronts");
constexpr int kSlotLoads = kRedBlocks / 64;
constexpr int kSlotsPerWave = kSlotLoads >= 16 ? 1 : 16 / kSlotLoads;
__device__ __forceinline__ void reduce_slots(const cpx<double>* __restrict__ part, int rhs, int cnt, cpx<double>* sums) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const cpx<double>* pr = part + (size_t)rhs * kPartSlots * kRedBlocks + lane;
  for (int s0 = wv; s0 < cnt; s0 += kSlotsPerWave * nw) {
    cpx<double> x[kSlotsPerWave][kSlotLoads];
#pragma unroll
    for (int q = 0; q < kSlotsPerWave; ++q) {
      const int sl = s0 + q * nw;
      const cpx<double>* p = pr + (size_t)(sl < cnt ? sl : s0) * kRedBlocks;
#pragma unroll
      for (int b = 0; b < kSlotLoads; ++b) x[q][b] = p[64 * b];
    }
#pragma unroll
    for (int q = 0; q < kSlotsPerWave; ++q) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int b = 0; b < kSlotLoads; ++b) {
        re += x[q][b].re;
        im += x[q][b].im;
      }
      re = wave_sum(re);
      im = wave_sum(im);
      const int sl = s0 + q * nw;
      if (lane == 0 && sl < cnt) sums[sl] = {re, im};
    }
  }
  lds_barrier();
}

// Givens state of one right-hand side staged in LDS by the finishing kernels.
struct GivensLds {
  cpx<double> cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1];
  cpx<double> col[kMaxRestart + 2];
};

// Commit Hessenberg column j given its unrotated entries raw[0..j+1] (in LDS):
// apply the previous Givens rotations (rotated column to L.col), form rotation j,
// rotate g and store the rotation and g in the state.  Single thread; the
// columns themselves are stored by store_column.  `iters`: the state's step count,
// read at kernel start (a global load here would stall the chain), incremented
// and stored.  Returns |g_{j+1}|.
__device__ double commit_column(KState& S, GivensLds& L, int j, const cpx<double>* raw, int& iters) {
  cpx<double>* col = L.col;
  // Rotation i mixes entries i and i+1.  The entry carried to the next rotation
  // stays in registers, and the operands of four rotations are loaded from LDS
  // at once (indices clamped in range), so the dependent chain waits for LDS once
  // per four steps.
  constexpr int U = 4;
  cpx<double> a = raw[0];
  for (int i0 = 0; i0 < j; i0 += U) {
    cpx<double> bb[U], cc[U], ss[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u < j ? i0 + u : j - 1;
      bb[u] = raw[i + 1];
      cc[u] = L.cs[i];
      ss[u] = L.sn[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + u >= j) break;
      const cpx<double> b = bb[u], c = cc[u], s = ss[u];
      // [conj(c) conj(s); -s c] applied to (a, b)
      col[i0 + u] = {c.re * a.re + c.im * a.im + s.re * b.re + s.im * b.im,
                     c.re * a.im - c.im * a.re + s.re * b.im - s.im * b.re};
      a = {-(s.re * a.re - s.im * a.im) + (c.re * b.re - c.im * b.im),
           -(s.re * a.im + s.im * a.re) + (c.re * b.im + c.im * b.re)};
    }
  }
  const double hn = raw[j + 1].re;   // the subdiagonal entry is real and >= 0
  const double aa = sqrt(cabs2(a));
  const double den = sqrt(aa * aa + hn * hn);
  cpx<double> c, s;
  if (den == 0.0) { c = {1.0, 0.0}; s = {0.0, 0.0}; }
  else if (aa == 0.0) { c = {0.0, 0.0}; s = {1.0, 0.0}; }
  else { c = {a.re / den, a.im / den}; s = {hn / den, 0.0}; }
  L.cs[j] = c;
  L.sn[j] = s;
  col[j] = {den, 0.0};
  col[j + 1] = {0.0, 0.0};
  const cpx<double> gj = L.g[j];
  L.g[j] = {c.re * gj.re + c.im * gj.im, c.re * gj.im - c.im * gj.re};   // conj(c) g_j
  L.g[j + 1] = {-s.re * gj.re, -s.re * gj.im};
  S.cs[j] = c;
  S.sn[j] = s;
  S.g[j] = L.g[j];
  S.g[j + 1] = L.g[j + 1];
  S.k = j + 1;
  S.iters = ++iters;
  return sqrt(cabs2(L.g[j + 1]));
}

// Make one lane's LDS writes visible to the rest of its wavefront.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Store committed column j (raw and rotated entries 0..j+1) in the state; the
// lanes of one wavefront share the entries.
__device__ __forceinline__ void store_column(KState& S, const GivensLds& L, int j, const cpx<double>* raw, int lane) {
  cpx<double>* hr = S.Hraw + (size_t)j * (kMaxRestart + 1);
  cpx<double>* hc = S.H + (size_t)j * (kMaxRestart + 1);
  for (int i = lane; i <= j + 1; i += 64) {
    hr[i] = raw[i];
    hc[i] = L.col[i];
  }
}

__device__ __forceinline__ void publish_stop(int* host_stop, int rhs, int v) {
  if (host_stop != nullptr) host_stop[rhs] = v;
}

// What the last block does with the sums.
enum DotsMode { kDotsFnorm = 0, kDotsCycle = 1, kDotsPlain = 2 };

struct DotsCtl {
  KState* state;
  int* skip_step;
  int* done;
  int* host_stop;
  int* host_done;
  int mode, j, restart;
  double rtol;
};

__device__ void dots_finalize(const DotsCtl& c, const cpx<double>* part, int rhs, int nvec) {
  __shared__ cpx<double> sums[kPartSlots];
  reduce_slots(part, rhs, nvec + 1, sums);
  if (threadIdx.x != 0) return;
  KState& S = c.state[rhs];
  if (c.mode == kDotsFnorm) {            // ||f|| once per solve; target = rtol ||f||
    S.fnorm = sqrt(sums[0].re);
    S.target = c.rtol * S.fnorm;
    S.iters = 0;
    S.cycles = 0;
    // a non-finite right-hand side stops at once, its residual marked NaN
    const bool finite = isfinite(S.fnorm);
    S.relres = !finite ? __builtin_nan("") : S.fnorm > 0.0 ? 1.0 : 0.0;
    c.done[rhs] = finite && S.fnorm > 0.0 ? 0 : 1;
    c.skip_step[rhs] = c.done[rhs];
    publish_stop(c.host_stop, rhs, c.skip_step[rhs]);
    publish_stop(c.host_done, rhs, c.done[rhs]);
  } else if (c.mode == kDotsPlain) {     // unpreconditioned norms of a left-preconditioned solve
    const double nrm = sqrt(sums[0].re);
    if (c.j == 0) {
      S.fnorm_plain = nrm;
    } else {
      // a non-finite norm on either side propagates as NaN (never reads as converged)
      const double fp = S.fnorm_plain;
      S.relres_plain = !(isfinite(fp) && isfinite(nrm)) ? __builtin_nan("") : fp > 0.0 ? nrm / fp : 0.0;
    }
  } else if (c.mode == kDotsCycle) {     // cycle start: beta = ||r||, residual test
    const double beta = sqrt(sums[0].re);
    S.beta = beta;
    S.relres = S.fnorm > 0.0 ? beta / S.fnorm : 0.0;
    S.stop_at = -1;
    if (!isfinite(beta)) {               // a non-finite residual (e.g. from the initial guess)
      S.relres = __builtin_nan("");
      c.done[rhs] = 1;
      c.skip_step[rhs] = 1;
    } else if (S.relres <= c.rtol || beta == 0.0) {
      c.done[rhs] = 1;
      c.skip_step[rhs] = 1;
    } else {
      S.cycles += 1;
      S.k = 0;
      for (int i = 0; i <= kMaxRestart; ++i) S.g[i] = {0.0, 0.0};
      S.g[0] = {beta, 0.0};
      c.skip_step[rhs] = 0;
    }
    publish_stop(c.host_stop, rhs, c.skip_step[rhs]);
    publish_stop(c.host_done, rhs, c.done[rhs]);
  }
}

// part[rhs][blk][0..nvec-1] = V_v^H w (partial), part[..][nvec] = ||w||^2 (partial);
// the last block of each right-hand side reduces them (see DotsMode).
__global__ __launch_bounds__(kRedThreads) void k_dots(const cpx<double>* __restrict__ V, size_t npts,
                                                       size_t vrs, const cpx<double>* __restrict__ w,
                                                       size_t wrs, int nvec, cpx<double>* __restrict__ part,
                                                       const int* __restrict__ skip, DotsCtl ctl) {
  const int rhs = blockIdx.y;
  if (skip != nullptr && skip[rhs] != 0) return;
  const cpx<double>* Vr = V + (size_t)rhs * vrs;
  const cpx<double>* wr = w + (size_t)rhs * wrs;
  cpx<double>* pr = part + (size_t)rhs * kPartSlots * kRedBlocks + blockIdx.x;
  const size_t stride = (size_t)kRedBlocks * kRedThreads;
  {
    cpx<double> nrm[1] = {{0.0, 0.0}};
    for (size_t i = (size_t)blockIdx.x * kRedThreads + threadIdx.x; i < npts; i += stride) {
      const cpx<double> a = wr[i];
      nrm[0].re += a.re * a.re + a.im * a.im;
    }
    block_reduce_write<1>(nrm, 1, pr + (size_t)nvec * kRedBlocks);
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
    block_reduce_write<kChunk>(acc, cnt, pr + (size_t)c0 * kRedBlocks);
  }
}

__global__ __launch_bounds__(1024) void k_dots_fin(const cpx<double>* __restrict__ part, DotsCtl ctl) {
  const int rhs = blockIdx.x;
  if (ctl.mode == kDotsCycle && ctl.done[rhs]) return;
  dots_finalize(ctl, part, rhs, 0);
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

// Arnoldi step j, one reduction over v_0..v_{j-1} (slots 0..j-1), u_j (slot j)
// and w = A u_j (slot j+1).  Partial-sum slots: [0, j) a = V^H u_j,
// [j, 2j) b = V^H w, 2j ||u_j||^2, 2j+1 u_j^H w, 2j+2 ||w||^2.

// Element-wise load of a complex value (keeps a conditional struct copy from
// becoming a private-memory temporary).
__device__ __forceinline__ cpx<double> ldc(const cpx<double>& p) { return {p.re, p.im}; }

// Hessenberg columns 0..j-2 staged in LDS, packed: column i (entries 0..i+1) at
// offset i (i + 3) / 2.
__device__ __forceinline__ int hpacked(int i) { return i * (i + 3) / 2; }
constexpr int kHPacked = kMaxRestart * (kMaxRestart + 3) / 2;
constexpr int kFinThreads = 1024;
constexpr int kHPrefetch = ((kMaxRestart - 1) * (kMaxRestart + 1) + kFinThreads - 1) / kFinThreads;

__device__ __forceinline__ void arnoldi_finalize(KState& S, const cpx<double>* part, int rhs, int j, int restart,
                                                 int* skip_step, int* host_stop) {
  __shared__ cpx<double> sums[kPartSlots];
  __shared__ cpx<double> zz[kMaxRestart + 1], hp[kMaxRestart + 1], raw[kMaxRestart + 2];
  __shared__ cpx<double> hsh[kHPacked];
  __shared__ GivensLds L;
  __shared__ double sh_sigma;
  __shared__ int sh_break;
  // Every load of the state this step reads (Givens rotations, g, the provisional
  // column, the finished Hessenberg columns but the last) is issued together with
  // the partial sums, so that their latencies overlap; they go to LDS afterwards.
  // (loads are unconditional, from clamped in-bounds indices, so that they stay
  // plain register loads; the unused values are dropped)
  const int t = threadIdx.x;
  const int tc = t < kMaxRestart ? t : 0, tg = t <= kMaxRestart ? t : 0;
  const cpx<double> rc = ldc(S.cs[tc]), rs = ldc(S.sn[tc]), rg = ldc(S.g[tg]), rh = ldc(S.hprov[tg]);
  cpx<double> hv[kHPrefetch];
  int hdst[kHPrefetch];
  const int ld = j + 1;            // columns 0..j-2, rows 0..j as a rectangle
#pragma unroll
  for (int r = 0; r < kHPrefetch; ++r) {
    const int e = t + kFinThreads * r;
    const int i = e / ld, k = e - i * ld;
    const bool use = i < j - 1 && k <= i + 1;
    hv[r] = ldc(S.Hraw[use ? (size_t)i * (kMaxRestart + 1) + k : 0]);
    hdst[r] = use ? hpacked(i) + k : -1;
  }
  const double target = S.target;
  int iters = S.iters;
  reduce_slots(part, rhs, 2 * j + 3, sums);   // ends with a barrier
  if (t < kMaxRestart) { L.cs[t] = rc; L.sn[t] = rs; }
  if (t <= kMaxRestart) { L.g[t] = rg; hp[t] = rh; }
#pragma unroll
  for (int r = 0; r < kHPrefetch; ++r)
    if (hdst[r] >= 0) hsh[hdst[r]] = hv[r];
  lds_barrier();
  const cpx<double>* a = sums;
  const cpx<double>* bv = sums + j;
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < 64) {
    // v_j = (u_j - V a) / sigma; column j-1 = (hprov_{j-1} + a, sigma)
    const double aa = wave_sum(lane < j ? cabs2(a[lane]) : 0.0);
    const double s2 = sums[2 * j].re - aa;
    const double sigma = s2 > 0.0 ? sqrt(s2) : 0.0;
    const int brk = !(sigma > 0.0);
    if (lane == 0) {
      sh_sigma = sigma;
      sh_break = brk;
    }
    if (j >= 1) {
      if (lane < j) raw[lane] = cadd(hp[lane], a[lane]);
      if (lane == 0) raw[j] = {sigma, 0.0};
      wave_lds_sync();
      double est = 0.0;
      if (lane == 0) est = commit_column(S, L, j - 1, raw, iters);
      wave_lds_sync();
      store_column(S, L, j - 1, raw, lane);
      if (lane == 0 && (brk || est <= target)) {   // the cycle ended with column j-1
        S.stop_at = j - 1;
        skip_step[rhs] = 1;
        publish_stop(host_stop, rhs, 1);
        sh_break = 1;
      }
    }
  }
  lds_barrier();
  if (sh_break) return;
  // z = Hraw[0..j][0..j-1] a, the expansion of A V a in v_0..v_j (column j-1 is
  // the one committed above, still in raw).  Sixteen lanes per row k, each over
  // every sixteenth term, then summed across the sixteen in a fixed order.
  {
    static_assert(kFinThreads >= 16 * (kMaxRestart + 1) - 16, "one 16-lane group per row of z");
    const int k = threadIdx.x >> 4, q = threadIdx.x & 15;
    cpx<double> acc = {0.0, 0.0};
    if (k <= j) {
      for (int i = (k > 0 ? k - 1 : 0) + q; i < j; i += 16)
        acc = cadd(acc, cmul(i < j - 1 ? hsh[hpacked(i) + k] : raw[k], a[i]));
    }
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) {
      acc.re += __shfl_xor(acc.re, off, 16);
      acc.im += __shfl_xor(acc.im, off, 16);
    }
    if (k <= j && q == 0) zz[k] = acc;
  }
  const double sigma = sh_sigma, isg = 1.0 / sigma;
  if (threadIdx.x < 64) {
    // p_j = v_j^H w
    cpx<double> t = {0.0, 0.0};
    if (lane < j) t = {a[lane].re * bv[lane].re + a[lane].im * bv[lane].im, a[lane].re * bv[lane].im - a[lane].im * bv[lane].re};
    const cpx<double> ab = {wave_sum(t.re), wave_sum(t.im)};
    if (lane == 0) raw[j] = cscale(csub(sums[2 * j + 1], ab), isg);
  }
  lds_barrier();
  // hprov_j = [V, v_j]^H A v_j = (p - z) / sigma (parallel over k)
  for (int k = threadIdx.x; k <= j; k += blockDim.x) {
    const cpx<double> pk = k < j ? bv[k] : raw[j];
    hp[k] = cscale(csub(pk, zz[k]), isg);
  }
  lds_barrier();
  // update coefficients: u_{j+1} = w/sigma - V cv - cu u_j, y = z/sigma + hprov_j
  const cpx<double> cu = cscale(cadd(cscale(zz[j], isg), hp[j]), isg);
  for (int k = threadIdx.x; k <= j; k += blockDim.x) {
    S.hprov[k] = hp[k];
    if (k < j) {
      const cpx<double> yk = cadd(cscale(zz[k], isg), hp[k]);
      S.cv[k] = csub(yk, cmul(cu, a[k]));
      S.av[k] = a[k];
    }
  }
  if (threadIdx.x >= 64) return;
  double zp = 0.0, z2 = 0.0, h2 = 0.0;
  if (lane <= j) {
    const cpx<double> pk = lane < j ? bv[lane] : raw[j];
    zp = zz[lane].re * pk.re + zz[lane].im * pk.im;
    z2 = cabs2(zz[lane]);
    h2 = cabs2(hp[lane]);
  }
  zp = wave_sum(zp);
  z2 = wave_sum(z2);
  h2 = wave_sum(h2);
  // from here on every lane of wave 0 computes the same values
  if (lane == 0) {
    S.cu = cu;
    S.inv_sigma = isg;
  }
  const double av2 = (sums[2 * j + 2].re - 2.0 * zp + z2) * isg * isg;   // ||A v_j||^2
  const double r2 = av2 - h2;
  const double rho = r2 > 0.0 ? sqrt(r2) : 0.0;
  // residual estimate with the provisional column j (operands of four rotations
  // loaded at once, as in commit_column)
  cpx<double> t0 = hp[0];
  for (int i0 = 0; i0 < j; i0 += 4) {
    cpx<double> xx[4], cc[4], ss[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u < j ? i0 + u : j - 1;
      xx[u] = hp[i + 1];
      cc[u] = L.cs[i];
      ss[u] = L.sn[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + u >= j) break;
      const cpx<double> x1 = xx[u], c = cc[u], s = ss[u];
      t0 = {-(s.re * t0.re - s.im * t0.im) + (c.re * x1.re - c.im * x1.im),
            -(s.re * t0.im + s.im * t0.re) + (c.re * x1.im + c.im * x1.re)};
    }
  }
  const double tt = sqrt(cabs2(t0));
  const double den = sqrt(tt * tt + rho * rho);
  const double est = den > 0.0 ? rho / den * sqrt(cabs2(L.g[j])) : 0.0;
  const bool breakdown = rho <= 1e-14 * sqrt(av2 > 0.0 ? av2 : 0.0);
  if (est <= target || breakdown || j + 1 >= restart) {
    // end the cycle with the provisional column j (its second projection would
    // change it by the loss of orthogonality only)
    if (lane <= j) raw[lane] = hp[lane];
    if (lane == 0) raw[j + 1] = {rho, 0.0};
    wave_lds_sync();
    if (lane == 0) commit_column(S, L, j, raw, iters);
    wave_lds_sync();
    store_column(S, L, j, raw, lane);
    if (lane == 0) {
      S.stop_at = j;
      skip_step[rhs] = 1;
      publish_stop(host_stop, rhs, 1);
    }
  }
}

// Block b of a right-hand side owns the contiguous point range
// [b*range, (b+1)*range), range = ceil(npts / kRedBlocks), and walks it in tiles
// of kDotsTile points: u_j and w of the tile are staged in LDS once (their norms
// and u_j^H w accumulated on the way), then wave q streams the basis vectors
// q, q + NW, q + 2 NW, ... over the tile, kDotsBatch loads in flight per lane,
// accumulating V_k^H u_j and V_k^H w in registers.  Every basis element is read
// once and every slot is owned by one wave (no block reduction for them).
constexpr int kDotsTile = 1024;
constexpr int kDotsBatch = 8;
constexpr int kDotsSlots = 8;   // basis vectors per wave: j <= NW * kDotsSlots

// Where the sweep takes w = A u_j from: the stored vector (slot j+1), or, fused
// with the right-preconditioned step, the stencil applied to z = Q u_j as each
// tile is staged (w is then also stored in slot j+1 for the update kernel; the
// separate stencil pass, its read of w and a launch are saved).
struct WStored {
  const cpx<double>* W;
  __device__ __forceinline__ cpx<double> operator()(size_t p) const { return W[p]; }
};
template <typename R, typename TI, int DIM>
struct WStencil {
  const cpx<TI>* z;
  const cpx<R>* coef;
  cpx<double>* W;
  int n0, n1, n2;
  R ih0, ih1, ih2;
  __device__ __forceinline__ cpx<double> operator()(size_t p) const {
    const cpx<double> w = cvt<double>(stencil_point<R, TI, DIM>(z, coef, p, n0, n1, n2, ih0, ih1, ih2));
    W[p] = w;
    return w;
  }
};

// The sweep of one block over its range of one right-hand side's basis Vr; pr:
// this block's partial-sum column.
template <int NW, typename WSrc>
__device__ __forceinline__ void arnoldi_dots_body(const cpx<double>* Vr, size_t npts, cpx<double>* pr, int j,
                                                  const WSrc& wsrc, int bx) {
  __shared__ cpx<double> su[kDotsTile], sw[kDotsTile];
  __shared__ double red[NW][6];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const cpx<double>* U = Vr + (size_t)j * npts;
  const size_t range = (npts + kRedBlocks - 1) / kRedBlocks;
  const size_t r0 = (size_t)bx * range;
  const size_t r1 = r0 + range < npts ? r0 + range : npts;
  cpx<double> acc[2 * kDotsSlots];
#pragma unroll
  for (int v = 0; v < 2 * kDotsSlots; ++v) acc[v] = {0.0, 0.0};
  double uu = 0.0, uwr = 0.0, uwi = 0.0, ww = 0.0;
  for (size_t t0 = r0; t0 < r1; t0 += kDotsTile) {
    const int n = (int)(r1 - t0 < (size_t)kDotsTile ? r1 - t0 : kDotsTile);
    for (int i = threadIdx.x; i < n; i += NW * 64) {
      const cpx<double> u = U[t0 + i], w = wsrc(t0 + i);
      su[i] = u;
      sw[i] = w;
      uu += u.re * u.re + u.im * u.im;
      uwr += u.re * w.re + u.im * w.im;     // conj(u) w
      uwi += u.re * w.im - u.im * w.re;
      ww += w.re * w.re + w.im * w.im;
    }
    __syncthreads();
#pragma unroll
    for (int sl = 0; sl < kDotsSlots; ++sl) {
      const int k = q + NW * sl;
      if (k >= j) break;
      const cpx<double>* vk = Vr + (size_t)k * npts + t0;
      for (int p0 = 0; p0 < n; p0 += 64 * kDotsBatch) {
        cpx<double> x[kDotsBatch];
        if (p0 + 64 * kDotsBatch <= n) {
#pragma unroll
          for (int b = 0; b < kDotsBatch; ++b) x[b] = vk[p0 + lane + 64 * b];
        } else {
#pragma unroll
          for (int b = 0; b < kDotsBatch; ++b) {
            const int p = p0 + lane + 64 * b;
            x[b] = p < n ? vk[p] : cpx<double>{0.0, 0.0};
          }
        }
#pragma unroll
        for (int b = 0; b < kDotsBatch; ++b) {
          int p = p0 + lane + 64 * b;
          p = p < n ? p : 0;   // x[b] is zero there
          const cpx<double> u = su[p], w = sw[p];
          acc[2 * sl].re += x[b].re * u.re + x[b].im * u.im;     // conj(v) u
          acc[2 * sl].im += x[b].re * u.im - x[b].im * u.re;
          acc[2 * sl + 1].re += x[b].re * w.re + x[b].im * w.im; // conj(v) w
          acc[2 * sl + 1].im += x[b].re * w.im - x[b].im * w.re;
        }
      }
    }
    __syncthreads();
  }
  // slots: a = V^H u_j at [0, j), b = V^H w at [j, 2j), then ||u_j||^2, u_j^H w, ||w||^2
#pragma unroll
  for (int sl = 0; sl < kDotsSlots; ++sl) {
    const int k = q + NW * sl;
    if (k >= j) break;
    const double ar = wave_sum(acc[2 * sl].re), ai = wave_sum(acc[2 * sl].im);
    const double br = wave_sum(acc[2 * sl + 1].re), bi = wave_sum(acc[2 * sl + 1].im);
    if (lane == 0) {
      pr[(size_t)k * kRedBlocks] = {ar, ai};
      pr[(size_t)(j + k) * kRedBlocks] = {br, bi};
    }
  }
  uu = wave_sum(uu);
  uwr = wave_sum(uwr);
  uwi = wave_sum(uwi);
  ww = wave_sum(ww);
  if (lane == 0) {
    red[q][0] = uu; red[q][1] = uwr; red[q][2] = uwi; red[q][3] = ww;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int w = 0; w < NW; ++w) { s0 += red[w][0]; s1 += red[w][1]; s2 += red[w][2]; s3 += red[w][3]; }
    pr[(size_t)(2 * j) * kRedBlocks] = {s0, 0.0};
    pr[(size_t)(2 * j + 1) * kRedBlocks] = {s1, s2};
    pr[(size_t)(2 * j + 2) * kRedBlocks] = {s3, 0.0};
  }
}

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_arnoldi_dots(const cpx<double>* __restrict__ V, size_t npts,
                                                          size_t vrs, cpx<double>* __restrict__ part,
                                                          const int* __restrict__ skip_step, int j) {
  const int rhs = blockIdx.y;
  if (skip_step[rhs]) return;
  const cpx<double>* Vr = V + (size_t)rhs * vrs;
  arnoldi_dots_body<NW>(Vr, npts, part + (size_t)rhs * kPartSlots * kRedBlocks + blockIdx.x, j,
                        WStored{Vr + (size_t)(j + 1) * npts}, blockIdx.x);
}

template <int NW, typename R, typename TI, int DIM>
__global__ __launch_bounds__(NW * 64) void k_arnoldi_dots_st(cpx<double>* V, size_t npts, size_t vrs,
                                                             cpx<double>* __restrict__ part,
                                                             const int* __restrict__ skip_step, int j,
                                                             const cpx<TI>* __restrict__ z, size_t z_rs,
                                                             const cpx<R>* __restrict__ coef, int n0, int n1,
                                                             int n2, R ih0, R ih1, R ih2) {
  const int rhs = blockIdx.y;
  if (skip_step[rhs]) return;
  cpx<double>* Vr = V + (size_t)rhs * vrs;
  arnoldi_dots_body<NW>(Vr, npts, part + (size_t)rhs * kPartSlots * kRedBlocks + blockIdx.x, j,
                        WStencil<R, TI, DIM>{z + (size_t)rhs * z_rs, coef, Vr + (size_t)(j + 1) * npts, n0, n1,
                                             n2, ih0, ih1, ih2}, blockIdx.x);
}

__global__ __launch_bounds__(kFinThreads) void k_arnoldi_fin(const cpx<double>* __restrict__ part, int* __restrict__ skip_step,
                                                      KState* state, int j, int restart, int* __restrict__ host_stop) {
  const int rhs = blockIdx.x;
  if (skip_step[rhs]) return;
  arnoldi_finalize(state[rhs], part, rhs, j, restart, skip_step, host_stop);
}

// slot j <- v_j = (u_j - V a) / sigma ; slot j+1 <- u_{j+1} = w / sigma - V cv - cu u_j.
// Runs for right-hand sides still in the cycle, and for the step that ended it.
// Each thread updates kUpdPts points (256 apart) per iteration and reads the
// basis in chunks of kUpdChunk vectors with every load issued: past v_{j-1} the
// index is clamped and the coefficient (zero in LDS) cancels the term.
constexpr int kUpdPts = 4;
constexpr int kUpdChunk = 4;

__device__ __forceinline__ void update_point(cpx<double>* U, cpx<double>* W, size_t i, cpx<double> sa,
                                             cpx<double> sc, double isg, cpx<double> cu) {
  const cpx<double> u = U[i], w = W[i];
  U[i] = cscale(csub(u, sa), isg);
  const cpx<double> cuu = cmul(cu, u);
  W[i] = {w.re * isg - sc.re - cuu.re, w.im * isg - sc.im - cuu.im};
}

__global__ __launch_bounds__(256) void k_arnoldi_update(cpx<double>* __restrict__ V, size_t npts, size_t vrs,
                                                        const KState* __restrict__ state,
                                                        const int* __restrict__ skip_step, int j) {
  __shared__ cpx<double> ca[kMaxRestart + 8], cc[kMaxRestart + 8];
  const int rhs = blockIdx.y;
  const KState& S = state[rhs];
  if (skip_step[rhs] && S.stop_at != j) return;
  for (int i = threadIdx.x; i < kMaxRestart + 8; i += blockDim.x) {
    ca[i] = i < j ? S.av[i] : cpx<double>{0.0, 0.0};
    cc[i] = i < j ? S.cv[i] : cpx<double>{0.0, 0.0};
  }
  __syncthreads();
  const double isg = S.inv_sigma;
  const cpx<double> cu = S.cu;
  cpx<double>* Vr = V + (size_t)rhs * vrs;
  cpx<double>* U = Vr + (size_t)j * npts;
  cpx<double>* W = Vr + (size_t)(j + 1) * npts;
  constexpr size_t span = 256 * kUpdPts;
  for (size_t base = (size_t)blockIdx.x * span; base < npts; base += (size_t)gridDim.x * span) {
    const size_t i0 = base + threadIdx.x;
    if (base + span <= npts) {
      cpx<double> sa[kUpdPts], sc[kUpdPts];
#pragma unroll
      for (int p = 0; p < kUpdPts; ++p) { sa[p] = {0.0, 0.0}; sc[p] = {0.0, 0.0}; }
      for (int v0 = 0; v0 < j; v0 += kUpdChunk) {
        cpx<double> x[kUpdChunk][kUpdPts];
#pragma unroll
        for (int t = 0; t < kUpdChunk; ++t) {
          const int k = v0 + t < j ? v0 + t : j - 1;
#pragma unroll
          for (int p = 0; p < kUpdPts; ++p) x[t][p] = Vr[(size_t)k * npts + i0 + 256 * p];
        }
#pragma unroll
        for (int t = 0; t < kUpdChunk; ++t) {
          const cpx<double> a = ca[v0 + t], c = cc[v0 + t];
#pragma unroll
          for (int p = 0; p < kUpdPts; ++p) {
            sa[p].re += a.re * x[t][p].re - a.im * x[t][p].im;
            sa[p].im += a.re * x[t][p].im + a.im * x[t][p].re;
            sc[p].re += c.re * x[t][p].re - c.im * x[t][p].im;
            sc[p].im += c.re * x[t][p].im + c.im * x[t][p].re;
          }
        }
      }
#pragma unroll
      for (int p = 0; p < kUpdPts; ++p) update_point(U, W, i0 + 256 * p, sa[p], sc[p], isg, cu);
    } else {
      for (int p = 0; p < kUpdPts; ++p) {
        const size_t i = i0 + 256 * p;
        if (i >= npts) break;
        cpx<double> sa = {0.0, 0.0}, sc = {0.0, 0.0};
        for (int k = 0; k < j; ++k) {
          const cpx<double> x = Vr[(size_t)k * npts + i], a = ca[k], c = cc[k];
          sa.re += a.re * x.re - a.im * x.im;
          sa.im += a.re * x.im + a.im * x.re;
          sc.re += c.re * x.re - c.im * x.im;
          sc.im += c.re * x.im + c.im * x.re;
        }
        update_point(U, W, i, sa, sc, isg, cu);
      }
    }
  }
}


// The update for FP64 2-D grids whose rows (512 to 2048 points) run the register
// transform: each workgroup updates whole rows of v_j and u_{j+1} (the same sums in
// the same order as k_arnoldi_update, over pairs of basis vectors) and, with u_{j+1}
// still in registers, transforms it along the rows into t: pass A of the next
// step's apply, whose launch and whose read of u_{j+1} are saved.
template <int N>
__global__ __launch_bounds__((RowCfg<double, N>::THREADS)) void k_arnoldi_update_rows(
    cpx<double>* __restrict__ V, size_t npts, size_t vrs, const KState* __restrict__ state,
    const int* __restrict__ skip_step, int j, cpx<double>* __restrict__ t, int rows,
    const cpx<double>* __restrict__ tw) {
  using C = RowCfg<double, N>;
  __shared__ cpx<double> ca[kMaxRestart + 8], cc[kMaxRestart + 8];
  __shared__ cpx<double> lds[C::LDS];
  const int rhs = blockIdx.y;
  const KState& S = state[rhs];
  if (skip_step[rhs] && S.stop_at != j) return;
  for (int i = threadIdx.x; i < kMaxRestart + 8; i += blockDim.x) {
    ca[i] = i < j ? S.av[i] : cpx<double>{0.0, 0.0};
    cc[i] = i < j ? S.cv[i] : cpx<double>{0.0, 0.0};
  }
  __syncthreads();
  const double isg = S.inv_sigma;
  const cpx<double> cu = S.cu;
  const int g = threadIdx.x / C::T;
  const int jj = rows_thread<double, N>((int)threadIdx.x % C::T);
  const int row = blockIdx.x * C::G + g;
  const bool act = row < rows;
  const size_t base = (size_t)(act ? row : 0) * N + jj;   // inactive rows load row 0 and store nothing
  cpx<double>* Vr = V + (size_t)rhs * vrs;
  cpx<double> sa[C::E], sc[C::E];
#pragma unroll
  for (int q = 0; q < C::E; ++q) { sa[q] = {0.0, 0.0}; sc[q] = {0.0, 0.0}; }
  constexpr int kPair = 2;
  for (int v0 = 0; v0 < j; v0 += kPair) {
    cpx<double> xv[kPair][C::E];
#pragma unroll
    for (int u = 0; u < kPair; ++u) {
      const int k = v0 + u < j ? v0 + u : j - 1;   // past v_{j-1} the coefficient is zero
#pragma unroll
      for (int q = 0; q < C::E; ++q) xv[u][q] = Vr[(size_t)k * npts + base + C::T * q];
    }
#pragma unroll
    for (int u = 0; u < kPair; ++u) {
      const cpx<double> a = ca[v0 + u], c = cc[v0 + u];
#pragma unroll
      for (int q = 0; q < C::E; ++q) {
        sa[q].re += a.re * xv[u][q].re - a.im * xv[u][q].im;
        sa[q].im += a.re * xv[u][q].im + a.im * xv[u][q].re;
        sc[q].re += c.re * xv[u][q].re - c.im * xv[u][q].im;
        sc[q].im += c.re * xv[u][q].im + c.im * xv[u][q].re;
      }
    }
  }
  cpx<double>* U = Vr + (size_t)j * npts;
  cpx<double>* W = Vr + (size_t)(j + 1) * npts;
  cpx<double> x[C::E];
#pragma unroll
  for (int q = 0; q < C::E; ++q) {
    const size_t i = base + C::T * q;
    const cpx<double> u = U[i], w = W[i];
    const cpx<double> cuu = cmul(cu, u);
    x[q] = {w.re * isg - sc[q].re - cuu.re, w.im * isg - sc[q].im - cuu.im};
    if (act) {
      U[i] = cscale(csub(u, sa[q]), isg);
      W[i] = x[q];
    }
  }
  fft_e<double, N, C::E, -1, true, 1, false, rows_swap<double, N>()>(x, lds + g * lds_elems<double>(N), jj, tw);
  if (act) {
    cpx<double>* dst = t + (size_t)rhs * npts + (size_t)row * N;
#pragma unroll
    for (int q = 0; q < C::E; ++q) dst[jj + C::T * q] = x[q];
  }
}

// The update of k_arnoldi_update for the grouped launches (bx, gx: this workgroup's
// index among the gx of one right-hand side).  The single-plan kernel keeps its own
// copy: its code, and so its rounding, stays exactly as it was.
__device__ __forceinline__ void arnoldi_update_body(cpx<double>* __restrict__ V, size_t npts, size_t vrs,
                                                    const KState* __restrict__ state,
                                                    const int* __restrict__ skip_step, int j, int rhs, int bx,
                                                    int gx) {
  __shared__ cpx<double> ca[kMaxRestart + 8], cc[kMaxRestart + 8];
  const KState& S = state[rhs];
  if (skip_step[rhs] && S.stop_at != j) return;
  for (int i = threadIdx.x; i < kMaxRestart + 8; i += blockDim.x) {
    ca[i] = i < j ? S.av[i] : cpx<double>{0.0, 0.0};
    cc[i] = i < j ? S.cv[i] : cpx<double>{0.0, 0.0};
  }
  __syncthreads();
  const double isg = S.inv_sigma;
  const cpx<double> cu = S.cu;
  cpx<double>* Vr = V + (size_t)rhs * vrs;
  cpx<double>* U = Vr + (size_t)j * npts;
  cpx<double>* W = Vr + (size_t)(j + 1) * npts;
  constexpr size_t span = 256 * kUpdPts;
  for (size_t base = (size_t)bx * span; base < npts; base += (size_t)gx * span) {
    const size_t i0 = base + threadIdx.x;
    if (base + span <= npts) {
      cpx<double> sa[kUpdPts], sc[kUpdPts];
#pragma unroll
      for (int p = 0; p < kUpdPts; ++p) { sa[p] = {0.0, 0.0}; sc[p] = {0.0, 0.0}; }
      for (int v0 = 0; v0 < j; v0 += kUpdChunk) {
        cpx<double> x[kUpdChunk][kUpdPts];
#pragma unroll
        for (int t = 0; t < kUpdChunk; ++t) {
          const int k = v0 + t < j ? v0 + t : j - 1;
#pragma unroll
          for (int p = 0; p < kUpdPts; ++p) x[t][p] = Vr[(size_t)k * npts + i0 + 256 * p];
        }
#pragma unroll
        for (int t = 0; t < kUpdChunk; ++t) {
          const cpx<double> a = ca[v0 + t], c = cc[v0 + t];
#pragma unroll
          for (int p = 0; p < kUpdPts; ++p) {
            sa[p].re += a.re * x[t][p].re - a.im * x[t][p].im;
            sa[p].im += a.re * x[t][p].im + a.im * x[t][p].re;
            sc[p].re += c.re * x[t][p].re - c.im * x[t][p].im;
            sc[p].im += c.re * x[t][p].im + c.im * x[t][p].re;
          }
        }
      }
#pragma unroll
      for (int p = 0; p < kUpdPts; ++p) update_point(U, W, i0 + 256 * p, sa[p], sc[p], isg, cu);
    } else {
      for (int p = 0; p < kUpdPts; ++p) {
        const size_t i = i0 + 256 * p;
        if (i >= npts) break;
        cpx<double> sa = {0.0, 0.0}, sc = {0.0, 0.0};
        for (int k = 0; k < j; ++k) {
          const cpx<double> x = Vr[(size_t)k * npts + i], a = ca[k], c = cc[k];
          sa.re += a.re * x.re - a.im * x.im;
          sa.im += a.re * x.im + a.im * x.re;
          sc.re += c.re * x.re - c.im * x.im;
          sc.im += c.re * x.im + c.im * x.re;
        }
        update_point(U, W, i, sa, sc, isg, cu);
      }
    }
  }
}


// y = R^{-1} g over the k finished columns (upper triangular back substitution),
// with R and g staged in LDS.
__global__ __launch_bounds__(256) void k_backsolve(KState* state, const int* done) {
  __shared__ cpx<double> R[kMaxRestart * kMaxRestart];
  __shared__ cpx<double> y[kMaxRestart];
  const int rhs = blockIdx.x;
  if (done[rhs]) return;
  KState& S = state[rhs];
  const int k = S.k;
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
    const int col = t / k, row = t % k;
    R[row * kMaxRestart + col] = row <= col ? S.H[(size_t)col * (kMaxRestart + 1) + row] : cpx<double>{0.0, 0.0};
  }
  for (int t = threadIdx.x; t < k; t += blockDim.x) y[t] = S.g[t];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    cpx<double> s = y[i];
    for (int l = i + 1; l < k; ++l) s = csub(s, cmul(R[i * kMaxRestart + l], y[l]));
    const cpx<double> d = R[i * kMaxRestart + i];
    const double dd = cabs2(d);
    y[i] = {(s.re * d.re + s.im * d.im) / dd, (s.im * d.re - s.re * d.im) / dd};
  }
  for (int i = 0; i < k; ++i) S.y[i] = y[i];
}

// out = sum_{i<k} y_i v_i
__global__ __launch_bounds__(256) void k_lincomb(const cpx<double>* __restrict__ V, size_t npts, size_t vrs,
                                                 const KState* __restrict__ state, cpx<double>* __restrict__ out,
                                                 size_t out_rs, int accumulate, const int* __restrict__ done) {
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
    if (accumulate) a = cadd(a, o[i]);
    o[i] = a;
  }
}

// v = b - v (the residual of a system whose right-hand side is given preconditioned)
__global__ __launch_bounds__(256) void k_rsub(const cpx<double>* __restrict__ b, size_t b_rs,
                                              cpx<double>* __restrict__ v, size_t v_rs, size_t n,
                                              const int* __restrict__ skip) {
  const int rhs = blockIdx.y;
  if (skip != nullptr && skip[rhs]) return;
  const cpx<double>* br = b + (size_t)rhs * b_rs;
  cpx<double>* vr = v + (size_t)rhs * v_rs;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    vr[i] = csub(br[i], vr[i]);
}

__global__ void k_fill_zero(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ---------------------------------------------------------------- plan set-up
__global__ __launch_bounds__(256) void k_media_scan(const double* __restrict__ c, const double* __restrict__ a,
                                                    const double* __restrict__ z, size_t n, double c0,
                                                    MediaScan* __restrict__ partial) {
  __shared__ double smin[256], smax[256], szmax[256];
  __shared__ int sbad[256], slay[256], svar[256];
  double cmin = INFINITY, cmax = -INFINITY, zmax = 0.0;
  int bad = 0, lay = 0, var = 0;
  const double a0 = a ? a[0] : 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double cv = c[i];
    bad |= !(cv > 0.0) || !isfinite(cv);
    cmin = fmin(cmin, cv);
    cmax = fmax(cmax, cv);
    if (a) {
      const double av = a[i];
      bad |= !(av >= 0.0) || !isfinite(av);
      var |= av != a0;
    }
    if (z) {
      const double zv = z[i];
      bad |= !(zv >= 0.0) || !isfinite(zv);
      zmax = fmax(zmax, zv);
      lay |= zv > 0.0 && fabs(cv - c0) > 1e-12 * c0;
    }
  }
  smin[threadIdx.x] = cmin; smax[threadIdx.x] = cmax; szmax[threadIdx.x] = zmax;
  sbad[threadIdx.x] = bad; slay[threadIdx.x] = lay; svar[threadIdx.x] = var;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      szmax[threadIdx.x] = fmax(szmax[threadIdx.x], szmax[threadIdx.x + w]);
      sbad[threadIdx.x] |= sbad[threadIdx.x + w];
      slay[threadIdx.x] |= slay[threadIdx.x + w];
      svar[threadIdx.x] |= svar[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    partial[blockIdx.x] = {smin[0], smax[0], szmax[0], a0, sbad[0], slay[0], svar[0], 0};
}

// Interpolation record of a point: real segment seg + t, or layer segment
// -(1 + j + t) (the inverse of decode_pos), by binary search in the nodes.
__device__ double encode_pos(const NodeTable& T, double c, double z) {
  if (T.Mt > 0 && z > 0.0) {
    const double zz = fmin(z, T.znode[T.Mt]);
    int lo = 0, hi = T.Mt;             // largest j with znode[j] <= zz, within [0, Mt-1]
    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (T.znode[mid] <= zz) lo = mid; else hi = mid; }
    const double t = (zz - T.znode[lo]) / (T.znode[lo + 1] - T.znode[lo]);
    return -(1.0 + lo + t);
  }
  if (T.M == 1) return 0.0;
  const double cc = fmin(fmax(c, T.cnode[0]), T.cnode[T.M - 1]);
  int lo = 0, hi = T.M - 1;            // largest s with cnode[s] <= cc, within [0, M-2]
  while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (T.cnode[mid] <= cc) lo = mid; else hi = mid; }
  const double t = (cc - T.cnode[lo]) / (T.cnode[lo + 1] - T.cnode[lo]);
  return lo + t;
}

// Position of a value among the second-axis nodes of a tensor scheme (damping a, or
// Im gamma for the layer tensor): r + u with weights 1-u on node r and u on node r+1
// (r in [0, Ma-2]).
__device__ double encode_damping(const NodeTable& T, double a) {
  const double aa = fmin(fmax(a, T.anode[0]), T.anode[T.Ma - 1]);
  int lo = 0, hi = T.Ma - 1;
  while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (T.anode[mid] <= aa) lo = mid; else hi = mid; }
  return lo + (aa - T.anode[lo]) / (T.anode[lo + 1] - T.anode[lo]);
}

__global__ __launch_bounds__(256) void k_plan_points(const double* __restrict__ c, const double* __restrict__ a,
                                                     const double* __restrict__ z, size_t n, NodeTable T,
                                                     double omega, double sih2, double* __restrict__ pos,
                                                     double* __restrict__ posa, cpx<double>* __restrict__ coef64,
                                                     cpx<float>* __restrict__ coef32) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double cv = c[i], zv = z ? z[i] : 0.0, av = a ? a[i] : 0.0;
    pos[i] = encode_pos(T, cv, T.has_layer ? zv : 0.0);
    if (T.Ma >= 2) posa[i] = encode_damping(T, T.second ? -cv * zv : av);
    const double gr = cv * cv * (1.0 - zv * zv), gi = -2.0 * cv * cv * zv;   // (c (1 - i zeta))^2
    const cpx<double> g2 = {gr, gi}, be = {omega * omega - 2.0 * gr * sih2, omega * av - 2.0 * gi * sih2};
    coef64[2 * i] = g2;
    coef64[2 * i + 1] = be;
    if (coef32) {
      coef32[2 * i] = {(float)g2.re, (float)g2.im};
      coef32[2 * i + 1] = {(float)be.re, (float)be.im};
    }
  }
}

__global__ __launch_bounds__(256) void k_row_masks(const double* __restrict__ pos, const double* __restrict__ posa,
                                                   int nl, NodeTable T, uint64_t* __restrict__ rowmask) {
  __shared__ uint64_t sm[256];
  const size_t row = blockIdx.x;
  uint64_t m = 0;
  for (int i = threadIdx.x; i < nl; i += 256) {
    int A, B;
    double t;
    const double pv = pos[row * nl + i];
    decode_pos(pv, T.M, T.Mt, T.mo, A, B, t);
    if (T.Ma >= 2) {   // the four nodes of the bilinear cell, where their weight is non-zero
      double pa = posa[row * nl + i];
      int r = (int)pa;
      r = r > T.Ma - 2 ? T.Ma - 2 : r;
      const double u = pa - (double)r;
      const double wc[2] = {A == B ? 1.0 : 1.0 - t, A == B ? 0.0 : t};
      const double wa[2] = {1.0 - u, u};
      const int nc[2] = {A, B};
      for (int q = 0; q < 2; ++q)
        for (int p = 0; p < 2; ++p)
          if (wc[p] != 0.0 && wa[q] != 0.0) m |= 1ull << (nc[p] + T.M * (r + q));
      continue;
    }
    if (T.order >= 2 && pv >= 0.0 && T.M > 1) {   // the whole Lagrange stencil
      int a = A - (T.order - 1) / 2;
      a = a < 0 ? 0 : (a > T.M - 1 - T.order ? T.M - 1 - T.order : a);
      for (int k = a; k <= a + T.order; ++k) m |= 1ull << k;
      continue;
    }
    if (A == B || t != 1.0) m |= 1ull << A;
    if (A != B && t != 0.0) m |= 1ull << B;
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] |= sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) rowmask[row] = sm[0];
}

hipError_t launch_media_scan(const double* c, const double* a, const double* zeta, size_t n, double c0,
                             MediaScan* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_media_scan, dim3(kScanBlocks), dim3(256), 0, st, c, a, zeta, n, c0, partial);
  return hipGetLastError();
}

hipError_t launch_plan_points(const double* c, const double* a, const double* zeta, size_t n, const NodeTable& T,
                              double omega, double sum_ih2, double* pos, double* posa, cpx<double>* coef64,
                              cpx<float>* coef32, hipStream_t st) {
  if (T.Ma >= 2 && posa == nullptr) return hipErrorInvalidValue;
  const size_t b = (n + 255) / 256;
  hipLaunchKernelGGL(k_plan_points, dim3((unsigned)(b < 4096 ? b : 4096)), dim3(256), 0, st, c, a, zeta, n, T, omega,
                     sum_ih2, pos, posa, coef64, coef32);
  return hipGetLastError();
}

hipError_t launch_row_masks(const double* pos, const double* posa, int nl, size_t rows, const NodeTable& T,
                            uint64_t* rowmask, hipStream_t st) {
  if (T.Ma >= 2 && posa == nullptr) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_row_masks, dim3((unsigned)rows), dim3(256), 0, st, pos, posa, nl, T, rowmask);
  return hipGetLastError();
}

static unsigned stream_blocks(size_t npts) {
  size_t b = (npts + 255) / 256;
  return (unsigned)(b < 2048 ? (b == 0 ? 1 : b) : 2048);
}

static DotsCtl dots_ctl(const KrylovArgs& a, int mode, int j, double rtol) {
  DotsCtl c;
  c.state = a.state;
  c.skip_step = a.skip_step;
  c.done = a.done;
  c.host_stop = a.host_stop;
  c.host_done = a.host_done;
  c.mode = mode;
  c.j = j;
  c.restart = a.restart;
  c.rtol = rtol;
  return c;
}

hipError_t launch_fnorm(const KrylovArgs& a, const cpx<double>* f, size_t frs, double rtol, hipStream_t st) {
  const DotsCtl c = dots_ctl(a, kDotsFnorm, 0, rtol);
  hipLaunchKernelGGL(k_dots, dim3(kRedBlocks, a.nrhs), dim3(kRedThreads), 0, st, a.V, a.npts, a.vrs, f, frs, 0,
                     a.part, (const int*)nullptr, c);
  hipLaunchKernelGGL(k_dots_fin, dim3(a.nrhs), dim3(1024), 0, st, (const cpx<double>*)a.part, c);
  return hipGetLastError();
}

hipError_t launch_plain_norm(const KrylovArgs& a, const cpx<double>* w, size_t wrs, int which, hipStream_t st) {
  const DotsCtl c = dots_ctl(a, kDotsPlain, which, 0.0);
  hipLaunchKernelGGL(k_dots, dim3(kRedBlocks, a.nrhs), dim3(kRedThreads), 0, st, a.V, a.npts, a.vrs, w, wrs, 0,
                     a.part, (const int*)nullptr, c);
  hipLaunchKernelGGL(k_dots_fin, dim3(a.nrhs), dim3(1024), 0, st, (const cpx<double>*)a.part, c);
  return hipGetLastError();
}

hipError_t launch_cycle_start(const KrylovArgs& a, double rtol, hipStream_t st) {
  const DotsCtl c = dots_ctl(a, kDotsCycle, 0, rtol);
  hipLaunchKernelGGL(k_dots, dim3(kRedBlocks, a.nrhs), dim3(kRedThreads), 0, st, a.V, a.npts, a.vrs, a.V, a.vrs, 0,
                     a.part, (const int*)a.done, c);
  hipLaunchKernelGGL(k_dots_fin, dim3(a.nrhs), dim3(1024), 0, st, (const cpx<double>*)a.part, c);
  return hipGetLastError();
}

hipError_t launch_scale_v0(const KrylovArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_v0, dim3(stream_blocks(a.npts), a.nrhs), dim3(256), 0, st, a.V, a.npts, a.vrs,
                     a.state, a.done);
  return hipGetLastError();
}

hipError_t launch_arnoldi_dots(const KrylovArgs& a, int j, hipStream_t st) {
  // four waves per block when there are 512 or more blocks per right-hand side
  // (two blocks per CU), else eight
  if (kRedBlocks >= 512 && j <= 4 * kDotsSlots)
    hipLaunchKernelGGL(k_arnoldi_dots<4>, dim3(kRedBlocks, a.nrhs), dim3(4 * 64), 0, st, a.V, a.npts, a.vrs,
                       a.part, (const int*)a.skip_step, j);
  else if (j <= 8 * kDotsSlots)
    hipLaunchKernelGGL(k_arnoldi_dots<8>, dim3(kRedBlocks, a.nrhs), dim3(8 * 64), 0, st, a.V, a.npts, a.vrs,
                       a.part, (const int*)a.skip_step, j);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_arnoldi_fin, dim3(a.nrhs), dim3(kFinThreads), 0, st, (const cpx<double>*)a.part, a.skip_step,
                     a.state, j, a.restart, a.host_stop);
  return hipGetLastError();
}

template <int NW, typename R, typename TI, int DIM>
static void dots_st_launch(const KrylovArgs& a, int j, const StencilArgs& s, hipStream_t st) {
  hipLaunchKernelGGL((k_arnoldi_dots_st<NW, R, TI, DIM>), dim3(kRedBlocks, a.nrhs), dim3(NW * 64), 0, st, a.V,
                     a.npts, a.vrs, a.part, (const int*)a.skip_step, j, (const cpx<TI>*)s.u, s.u_rs,
                     (const cpx<R>*)s.coef, s.n[0], s.n[1], s.dim == 3 ? s.n[2] : 1, (R)s.ih2[0], (R)s.ih2[1],
                     (R)s.ih2[2]);
}

template <int NW>
static hipError_t dots_st_dispatch(const KrylovArgs& a, int j, const StencilArgs& s, hipStream_t st) {
  if (s.kind == 0 && s.dim == 2) dots_st_launch<NW, double, double, 2>(a, j, s, st);
  else if (s.kind == 0 && s.dim == 3) dots_st_launch<NW, double, double, 3>(a, j, s, st);
  else if (s.kind == 2 && s.dim == 2) dots_st_launch<NW, float, float, 2>(a, j, s, st);
  else if (s.kind == 2 && s.dim == 3) dots_st_launch<NW, float, float, 3>(a, j, s, st);
  else return hipErrorInvalidValue;
  return hipSuccess;
}

hipError_t launch_arnoldi_dots_stencil(const KrylovArgs& a, int j, const StencilArgs& s, hipStream_t st) {
  hipError_t e;
  if (kRedBlocks >= 512 && j <= 4 * kDotsSlots) e = dots_st_dispatch<4>(a, j, s, st);
  else if (j <= 8 * kDotsSlots) e = dots_st_dispatch<8>(a, j, s, st);
  else return hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_arnoldi_fin, dim3(a.nrhs), dim3(kFinThreads), 0, st, (const cpx<double>*)a.part, a.skip_step,
                     a.state, j, a.restart, a.host_stop);
  return hipGetLastError();
}

// Rows of 512, 1024 and 2048 points.  Rows of 256 points (one workgroup per eight
// rows: a quarter of the plain update's workgroups on a 256^2 grid) measured no
// faster: 256^2 FP64 solve 4.82 -> 4.85 ms, 512^2 4.44 -> 4.38 ms.
bool update_rows_fits(int real_kind, int dim, int n_last) {
  return real_kind == 0 && dim == 2 && (n_last == 512 || n_last == 1024 || n_last == 2048);
}

hipError_t launch_arnoldi_update_rows(const KrylovArgs& a, int j, void* t, int n_last, const void* tw,
                                      hipStream_t st) {
  const int rows = (int)(a.npts / (size_t)n_last);
  auto go = [&](auto kern, int G, int threads) {
    hipLaunchKernelGGL(kern, dim3((unsigned)((rows + G - 1) / G), a.nrhs), dim3(threads), 0, st, a.V, a.npts, a.vrs,
                       (const KState*)a.state, (const int*)a.skip_step, j, (cpx<double>*)t, rows,
                       (const cpx<double>*)tw);
  };
  if (n_last == 512) go(k_arnoldi_update_rows<512>, RowCfg<double, 512>::G, RowCfg<double, 512>::THREADS);
  else if (n_last == 1024) go(k_arnoldi_update_rows<1024>, RowCfg<double, 1024>::G, RowCfg<double, 1024>::THREADS);
  else if (n_last == 2048) go(k_arnoldi_update_rows<2048>, RowCfg<double, 2048>::G, RowCfg<double, 2048>::THREADS);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_arnoldi_update(const KrylovArgs& a, int j, hipStream_t st) {
  const size_t ub = (a.npts + 256 * kUpdPts - 1) / (256 * kUpdPts);
  hipLaunchKernelGGL(k_arnoldi_update, dim3((unsigned)(ub < 1024 ? ub : 1024), a.nrhs), dim3(256), 0, st, a.V, a.npts, a.vrs,
                     a.state, a.skip_step, j);
  return hipGetLastError();
}

hipError_t launch_backsolve(const KrylovArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_backsolve, dim3(a.nrhs), dim3(256), 0, st, a.state, a.done);
  return hipGetLastError();
}

hipError_t launch_lincomb(const KrylovArgs& a, cpx<double>* out, size_t out_rs, bool accumulate, hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb, dim3(stream_blocks(a.npts), a.nrhs), dim3(256), 0, st, a.V, a.npts, a.vrs,
                     a.state, out, out_rs, accumulate ? 1 : 0, a.done);
  return hipGetLastError();
}

hipError_t launch_rsub(const cpx<double>* b, size_t b_rs, cpx<double>* v, size_t v_rs, size_t n, int nrhs,
                       const int* skip, hipStream_t st) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rsub, dim3(stream_blocks(n), nrhs), dim3(256), 0, st, b, b_rs, v, v_rs, n, skip);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3(stream_blocks(n)), dim3(256), 0, st, (uint32_t*)p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- grouped steps
// One launch per pass over several sessions of different grids and media (FP32
// preconditioner, right preconditioning, one right-hand side each): the member
// tables travel in the kernel arguments, each workgroup finds its member from the
// block offsets and runs the same body as the member's own kernel, with the same
// workgroup shape, so the results are bitwise those of the member's own step.
// Line lengths: 256-1024 on 2-D grids, 128-512 on 3-D grids.
template <typename D>
struct GroupArgs {
  int count;
  D m[kMaxGroup];
};

template <typename D>
__device__ __forceinline__ int group_member_of(const GroupArgs<D>& a) {
  int q = 0;
  while (q + 1 < a.count && (int)blockIdx.x >= a.m[q + 1].block0) ++q;
  return q;
}

constexpr int group_rows_lds() {
  return std::max({RowCfg<float, 128>::LDS, RowCfg<float, 256>::LDS, RowCfg<float, 512>::LDS,
                   RowCfg<float, 1024>::LDS});
}
constexpr int group_cols_lds() {
  return std::max({ColsCfg<float, 128, 1>::LDS, ColsCfg<float, 256, 1>::LDS, ColsCfg<float, 512, 1>::LDS,
                   ColsCfg<float, 1024, 1>::LDS, ColsCfg<float, 128, 0>::LDS, ColsCfg<float, 256, 0>::LDS,
                   ColsCfg<float, 512, 0>::LDS});
}
constexpr int group_cols_smask() {
  return std::max({cols_smask_words<float, 128, 1>(), cols_smask_words<float, 256, 1>(),
                   cols_smask_words<float, 512, 1>(), cols_smask_words<float, 1024, 1>()});
}
constexpr int group_comb_lds() {
  return std::max({WaveLine<float, 256>::LDS, WaveLine<float, 512>::LDS, WaveLine<float, 1024>::LDS,
                   combine_lds_elems<float, 128, 1>()});
}
static_assert(RowCfg<float, 128>::THREADS == 256 && RowCfg<float, 1024>::THREADS == 256, "grouped pass A shape");
static_assert(ColsCfg<float, 128, 1>::THREADS == 256 && ColsCfg<float, 1024, 1>::THREADS == 256 &&
                  ColsCfg<float, 128, 0>::THREADS == 256 && ColsCfg<float, 512, 0>::THREADS == 256,
              "grouped column pass shape");
static_assert(CombCfg<float, 128>::THREADS == 64, "grouped combine shape");

struct GRowsDesc {
  const cpx<double>* in;
  cpx<float>* out;
  const cpx<float>* tw;
  const int* skip;
  int rows, n, block0;
};

__global__ __launch_bounds__(256) void k_group_rows_fwd(const GroupArgs<GRowsDesc> a) {
  __shared__ cpx<float> lds[group_rows_lds()];
  const GRowsDesc& d = a.m[group_member_of(a)];
  if (d.skip[0] != 0) return;
  const int bx = (int)blockIdx.x - d.block0;
  switch (d.n) {
    case 128: rows_fwd_body<float, double, 128>(d.in, d.out, d.rows, 0, 0, d.tw, bx, 0, lds); break;
    case 256: rows_fwd_body<float, double, 256>(d.in, d.out, d.rows, 0, 0, d.tw, bx, 0, lds); break;
    case 512: rows_fwd_body<float, double, 512>(d.in, d.out, d.rows, 0, 0, d.tw, bx, 0, lds); break;
    case 1024: rows_fwd_body<float, double, 1024>(d.in, d.out, d.rows, 0, 0, d.tw, bx, 0, lds); break;
    default: break;
  }
}

struct GColsDesc {
  const cpx<float>* in;
  cpx<float>* out;
  const cpx<float>* tw;
  const int* skip;
  const double* lam_ax;
  const double* lam_in;
  const NodeConst* nodes;
  const uint16_t* store_mask;
  const uint8_t* slab_need;
  size_t in_rs, out_rs, in_fs, out_fs;
  double scale;
  int S, nfields, K, n, gx, gy, block0;
};

template <int DIR, int MODE>
__global__ __launch_bounds__(256) void k_group_cols(const GroupArgs<GColsDesc> a) {
  __shared__ cpx<float> lds[group_cols_lds()];
  __shared__ uint16_t smask[group_cols_smask()];
  const GColsDesc& d = a.m[group_member_of(a)];
  const int b = (int)blockIdx.x - d.block0;
  const int bx = b % d.gx, by = (b / d.gx) % d.gy, bz = b / (d.gx * d.gy);
#define HP_GCOLS(NN)                                                                                              \
  cols_body<float, float, NN, DIR, MODE>(d.in, d.out, d.S, d.nfields, d.in_rs, d.out_rs, d.in_fs, d.out_fs, d.tw, \
                                         d.skip, d.lam_ax, d.lam_in, d.nodes, d.K, d.scale, d.store_mask,        \
                                         d.slab_need, bx, by, bz, d.gx, d.gy, lds, smask)
  switch (d.n) {
    case 128: HP_GCOLS(128); break;
    case 256: HP_GCOLS(256); break;
    case 512: HP_GCOLS(512); break;
    case 1024:
      if constexpr (MODE == 1) HP_GCOLS(1024);
      break;
    default: break;
  }
#undef HP_GCOLS
}

struct GCombDesc {
  const cpx<float>* fields;
  const double* pos;
  const uint64_t* grpmask;
  const uint64_t* rowmask;
  cpx<float>* out;
  const cpx<float>* tw;
  const int* skip;
  const double* lag;
  const double* posa;
  size_t fs, frs;
  int rows, K, M, Mt, mo, ord, Ma, n, im, block0;
};

template <int IM>
__device__ __forceinline__ void group_combine_im(const GCombDesc& d, int bx, cpx<float>* lds, double* slag) {
#define HP_GCOMB_WAVE(NN)                                                                                           \
  comb_wave_body<float, float, NN, false, IM, 1>(d.fields, d.fs, d.frs, d.pos, d.rowmask, d.out, 0, d.rows, d.M, \
                                                 d.Mt, d.mo, d.tw, d.skip, d.ord, d.lag, d.posa, d.Ma, bx, 0, lds, \
                                                 slag)
  switch (d.n) {
    case 128:
      rows_combine_body<float, float, 128, false, IM, 1>(d.fields, d.fs, d.frs, d.pos, d.grpmask, d.rowmask, d.out, 0,
                                                         d.rows, d.K, d.M, d.Mt, d.mo, d.tw, d.skip, d.ord, d.lag,
                                                         d.posa, d.Ma, bx, 0, lds, slag);
      break;
    case 256: HP_GCOMB_WAVE(256); break;
    case 512: HP_GCOMB_WAVE(512); break;
    case 1024: HP_GCOMB_WAVE(1024); break;
    default: break;
  }
#undef HP_GCOMB_WAVE
}

// one launch per interpolation mode present among the members
template <int IM>
__global__ __launch_bounds__(64, 2) void k_group_combine(const GroupArgs<GCombDesc> a) {
  __shared__ cpx<float> lds[group_comb_lds()];
  __shared__ double slag[IM == kInterpLagrange ? kLagTable : 1];
  const GCombDesc& d = a.m[group_member_of(a)];
  group_combine_im<IM>(d, (int)blockIdx.x - d.block0, lds, slag);
}

// w = P_N z with the 2-D or the 3-D stencil chosen at run time (the same per-point
// arithmetic as the stencil pass, so w is bitwise the same)
struct WStencilAny {
  const cpx<float>* z;
  const cpx<float>* coef;
  cpx<double>* W;
  int dim, n0, n1, n2;
  float ih0, ih1, ih2;
  __device__ __forceinline__ cpx<double> operator()(size_t p) const {
    const cpx<float> v = dim == 2 ? stencil_point<float, float, 2>(z, coef, p, n0, n1, n2, ih0, ih1, ih2)
                                  : stencil_point<float, float, 3>(z, coef, p, n0, n1, n2, ih0, ih1, ih2);
    const cpx<double> w = cvt<double>(v);
    W[p] = w;
    return w;
  }
};

struct GDotsDesc {
  cpx<double>* V;
  cpx<double>* part;
  const int* skip;
  const cpx<float>* z;
  const cpx<float>* coef;
  size_t npts;
  float ih0, ih1, ih2;
  int j, dim, n0, n1, n2, block0;
};

__global__ __launch_bounds__(4 * 64) void k_group_dots(const GroupArgs<GDotsDesc> a) {
  const GDotsDesc& d = a.m[group_member_of(a)];
  if (d.skip[0] != 0) return;
  const int bx = (int)blockIdx.x - d.block0;
  arnoldi_dots_body<4>(d.V, d.npts, d.part + bx, d.j,
                       WStencilAny{d.z, d.coef, d.V + (size_t)(d.j + 1) * d.npts, d.dim, d.n0, d.n1, d.n2, d.ih0,
                                   d.ih1, d.ih2},
                       bx);
}

struct GFinDesc {
  const cpx<double>* part;
  int* skip;
  KState* state;
  int* host_stop;
  int j, restart;
};

__global__ __launch_bounds__(kFinThreads) void k_group_fin(const GroupArgs<GFinDesc> a) {
  const GFinDesc& d = a.m[blockIdx.x];
  if (d.skip[0] != 0) return;
  arnoldi_finalize(d.state[0], d.part, 0, d.j, d.restart, d.skip, d.host_stop);
}

struct GUpdDesc {
  cpx<double>* V;
  const KState* state;
  const int* skip;
  size_t npts;
  int j, gx, block0;
};

__global__ __launch_bounds__(256) void k_group_update(const GroupArgs<GUpdDesc> a) {
  const GUpdDesc& d = a.m[group_member_of(a)];
  arnoldi_update_body(d.V, d.npts, 0, d.state, d.skip, d.j, 0, (int)blockIdx.x - d.block0, d.gx);
}

static bool group_line_ok(int dim, int n) {
  return is_pow2_len(n) && (dim == 2 ? (n >= 256 && n <= 1024) : (n >= 128 && n <= 512));
}

bool group_member_ok(const GroupMember& m) {
  if ((m.dim != 2 && m.dim != 3) || m.K < 1 || m.K > kMaxNodes || m.j < 0 || m.j >= m.restart ||
      m.restart > 4 * kDotsSlots)
    return false;
  for (int d = 0; d < m.dim; ++d)
    if (!group_line_ok(m.dim, m.n[d])) return false;
  return true;
}

static int group_rows_per_block(int n) {
  switch (n) {
    case 128: return RowCfg<float, 128>::G;
    case 256: return RowCfg<float, 256>::G;
    case 512: return RowCfg<float, 512>::G;
    default: return RowCfg<float, 1024>::G;
  }
}
static int group_cols_tc(int n, int mode) {
  switch (n) {
    case 128: return mode == 1 ? ColsCfg<float, 128, 1>::TC : ColsCfg<float, 128, 0>::TC;
    case 256: return mode == 1 ? ColsCfg<float, 256, 1>::TC : ColsCfg<float, 256, 0>::TC;
    case 512: return mode == 1 ? ColsCfg<float, 512, 1>::TC : ColsCfg<float, 512, 0>::TC;
    default: return ColsCfg<float, 1024, 1>::TC;
  }
}

hipError_t launch_group_step(const GroupMember* m, int count, hipStream_t st) {
  if (count < 1 || count > kMaxGroup) return hipErrorInvalidValue;
  for (int q = 0; q < count; ++q)
    if (!group_member_ok(m[q])) return hipErrorInvalidValue;
  // pass A: forward transform of u_j along the contiguous axis
  {
    GroupArgs<GRowsDesc> A{};
    A.count = count;
    int blocks = 0;
    for (int q = 0; q < count; ++q) {
      const int nl = m[q].n[m[q].dim - 1];
      const int rows = (int)(m[q].npts / nl);
      A.m[q] = GRowsDesc{m[q].V + (size_t)m[q].j * m[q].npts, (cpx<float>*)m[q].t,
                         (const cpx<float>*)m[q].tw[m[q].dim - 1], m[q].skip_step, rows, nl, blocks};
      blocks += (rows + group_rows_per_block(nl) - 1) / group_rows_per_block(nl);
    }
    hipLaunchKernelGGL(k_group_rows_fwd, dim3(blocks), dim3(256), 0, st, A);
  }
  // middle-axis pass of the 3-D members: forward on t (A'), or inverse on the node fields (M)
  auto middle = [&](int dir) -> hipError_t {
    GroupArgs<GColsDesc> C{};
    int blocks = 0, c = 0;
    for (int q = 0; q < count; ++q) {
      if (m[q].dim != 3) continue;
      const int n1 = m[q].n[1], S = m[q].n[2], tc = group_cols_tc(n1, 0);
      const int nf = dir < 0 ? 1 : m[q].K;
      GColsDesc d{};
      d.in = (const cpx<float>*)(dir < 0 ? m[q].t : m[q].fields);
      d.out = (cpx<float>*)(dir < 0 ? m[q].t : m[q].fields);
      d.tw = (const cpx<float>*)m[q].tw[1];
      d.skip = m[q].skip_step;
      d.slab_need = dir < 0 ? nullptr : m[q].slab_need;
      d.in_rs = d.out_rs = (size_t)nf * m[q].npts;
      d.in_fs = d.out_fs = m[q].npts;
      d.S = S;
      d.nfields = nf;
      d.n = n1;
      d.gx = (S + tc - 1) / tc;
      d.gy = m[q].n[0];
      d.block0 = blocks;
      blocks += d.gx * d.gy * nf;
      C.m[c++] = d;
    }
    C.count = c;
    if (c == 0) return hipSuccess;
    if (dir < 0) hipLaunchKernelGGL((k_group_cols<-1, 0>), dim3(blocks), dim3(256), 0, st, C);
    else hipLaunchKernelGGL((k_group_cols<+1, 0>), dim3(blocks), dim3(256), 0, st, C);
    return hipGetLastError();
  };
  hipError_t e;
  if ((e = middle(-1)) != hipSuccess) return e;
  // pass B: forward along axis 0, K symbol multiplies and inverse transforms
  {
    GroupArgs<GColsDesc> B{};
    B.count = count;
    int blocks = 0;
    for (int q = 0; q < count; ++q) {
      const int n0 = m[q].n[0], S = (int)(m[q].npts / n0), tc = group_cols_tc(n0, 1);
      GColsDesc d{};
      d.in = (const cpx<float>*)m[q].t;
      d.out = (cpx<float>*)m[q].fields;
      d.tw = (const cpx<float>*)m[q].tw[0];
      d.skip = m[q].skip_step;
      d.lam_ax = m[q].lam_ax;
      d.lam_in = m[q].lam_in;
      d.nodes = m[q].nodes;
      d.store_mask = m[q].store_mask;
      d.slab_need = m[q].slab_need;
      d.in_rs = m[q].npts;
      d.out_rs = m[q].npts * (size_t)m[q].K;
      d.in_fs = d.out_fs = m[q].npts;
      d.scale = m[q].scale;
      d.S = S;
      d.nfields = 1;
      d.K = m[q].K;
      d.n = n0;
      d.gx = (S + tc - 1) / tc;
      d.gy = m[q].ng_b > 0 ? std::min(m[q].K, m[q].ng_b) : std::max(1, std::min(m[q].K, (512 + d.gx - 1) / d.gx));
      d.block0 = blocks;
      blocks += d.gx * d.gy;
      B.m[q] = d;
    }
    hipLaunchKernelGGL((k_group_cols<-1, 1>), dim3(blocks), dim3(256), 0, st, B);
  }
  if ((e = middle(+1)) != hipSuccess) return e;
  // pass C: inverse along the contiguous axis and the weighted sum into z
  for (int im = kInterpLinear; im <= kInterpBilinear; ++im) {
    GroupArgs<GCombDesc> Cb{};
    int blocks = 0, c = 0;
    for (int q = 0; q < count; ++q) {
      if (m[q].interp != im) continue;
      const int nl = m[q].n[m[q].dim - 1];
      const int rows = (int)(m[q].npts / nl);
      GCombDesc d{};
      d.fields = (const cpx<float>*)m[q].fields;
      d.pos = m[q].pos;
      d.grpmask = m[q].grpmask;
      d.rowmask = m[q].rowmask;
      d.out = (cpx<float>*)m[q].z;
      d.tw = (const cpx<float>*)m[q].tw[m[q].dim - 1];
      d.skip = m[q].skip_step;
      d.lag = m[q].lag;
      d.posa = m[q].posa;
      d.fs = m[q].npts;
      d.frs = m[q].npts * (size_t)m[q].K;
      d.rows = rows;
      d.K = m[q].K;
      d.M = m[q].M;
      d.Mt = m[q].Mt;
      d.mo = m[q].mo;
      d.ord = m[q].order;
      d.Ma = m[q].Ma;
      d.n = nl;
      d.im = m[q].interp;
      d.block0 = blocks;
      blocks += nl == 128 ? (rows + CombCfg<float, 128>::G - 1) / CombCfg<float, 128>::G : rows;
      Cb.m[c++] = d;
    }
    Cb.count = c;
    if (c == 0) continue;
    if (im == kInterpLagrange) hipLaunchKernelGGL(k_group_combine<kInterpLagrange>, dim3(blocks), dim3(64), 0, st, Cb);
    else if (im == kInterpBilinear) hipLaunchKernelGGL(k_group_combine<kInterpBilinear>, dim3(blocks), dim3(64), 0, st, Cb);
    else hipLaunchKernelGGL(k_group_combine<kInterpLinear>, dim3(blocks), dim3(64), 0, st, Cb);
  }
  // w = P_N z with the dot products of the step, then the finishing kernel and the update
  {
    GroupArgs<GDotsDesc> D{};
    GroupArgs<GFinDesc> F{};
    GroupArgs<GUpdDesc> U{};
    D.count = F.count = U.count = count;
    int ublocks = 0;
    for (int q = 0; q < count; ++q) {
      const GroupMember& g = m[q];
      D.m[q] = GDotsDesc{g.V, g.part, g.skip_step, (const cpx<float>*)g.z, (const cpx<float>*)g.coef32, g.npts,
                         (float)g.ih2[0], (float)g.ih2[1], (float)g.ih2[2], g.j, g.dim, g.n[0], g.n[1],
                         g.dim == 3 ? g.n[2] : 1, q * kRedBlocks};
      F.m[q] = GFinDesc{g.part, g.skip_step, g.state, g.host_stop, g.j, g.restart};
      const size_t ub = (g.npts + 256 * kUpdPts - 1) / (256 * kUpdPts);
      const int gx = (int)(ub < 1024 ? ub : 1024);
      U.m[q] = GUpdDesc{g.V, g.state, g.skip_step, g.npts, g.j, gx, ublocks};
      ublocks += gx;
    }
    hipLaunchKernelGGL(k_group_dots, dim3(count * kRedBlocks), dim3(4 * 64), 0, st, D);
    hipLaunchKernelGGL(k_group_fin, dim3(count), dim3(kFinThreads), 0, st, F);
    hipLaunchKernelGGL(k_group_update, dim3(ublocks), dim3(256), 0, st, U);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- static scratch
// Apply workspace of hp_apply_precond_static: a file-scope device array that every
// GPU the library runs on holds from module load to process exit.  Host code never
// uses the array's name as an address (on the host it names a stand-in): the
// device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept here.
static __device__ __align__(256) unsigned char scratch[HP_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t static_scratch(void** out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess) return e;
    if (ptr == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace hp
