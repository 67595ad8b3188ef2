// Internal declarations shared by the kernels (hp_kernels.hip) and the host
// side of the library (hp_api.cpp).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/helmpre.h"
#include "hp_fft.h"

namespace hp {

// Symbol constants of one node: q_n(lambda) = 1 / (A_n - g_n lambda) with
// A_n = omega^2 + i omega ahat_n and g_n = gamma_n^2 (Eqn. 021 with gamma).
struct NodeConst {
  double are, aim, gre, gim;
};

constexpr int kMaxNodes = 64;
constexpr int kMaxRestart = 64;

// Krylov state of one right-hand side, resident on the device.
// Arnoldi with classical Gram-Schmidt and lagged reorthogonalisation: step j
// applies the operator to the provisional vector u_j (projected once), and one
// reduction gives both the second projection of u_j (which finalises v_j and
// Hessenberg column j-1) and the projections of A u_j (which give column j).
struct KState {
  cpx<double> H[(kMaxRestart + 1) * kMaxRestart];     // rotated (R of the QR), column-major, ld kMaxRestart+1
  cpx<double> Hraw[(kMaxRestart + 1) * kMaxRestart];  // Hessenberg columns before rotation
  cpx<double> cs[kMaxRestart], sn[kMaxRestart];
  cpx<double> g[kMaxRestart + 1];
  cpx<double> y[kMaxRestart];
  cpx<double> hprov[kMaxRestart + 1];  // provisional column of the last step
  cpx<double> cv[kMaxRestart + 1];     // update coefficients on v_0..v_{j-1}
  cpx<double> av[kMaxRestart + 1];     // second-projection coefficients a of u_j
  cpx<double> cu;                      // update coefficient on u_j
  double fnorm, target, beta, inv_sigma, relres;
  double fnorm_plain, relres_plain;   // ||f|| and ||f - P x|| / ||f|| (left-preconditioned solves)
  int k;        // columns finished in the current cycle
  int stop_at;  // step at which the current cycle ends (-1: not yet)
  int iters;    // Arnoldi steps in total
  int cycles;
  int pad_[4];
};

#ifndef HP_RED_THREADS
#define HP_RED_THREADS 512
#endif
#ifndef HP_RED_BLOCKS
#define HP_RED_BLOCKS 512
#endif
constexpr int kRedThreads = HP_RED_THREADS;  // threads per block of the reduction kernels
constexpr int kRedBlocks = HP_RED_BLOCKS;    // blocks per right-hand side (fixed: deterministic sums)
constexpr int kPartSlots = 2 * kMaxRestart + 4;

// Mixed-radix lines (N = 2^a 3^b 5^c, not a power of two): stage radices in
// order, threads per line and (column passes) lines per workgroup.  A thread
// holds at most E elements of a line: kGenRowE in pass A, gen_e<R>() in the
// column passes and in pass C.
constexpr int kGenRowE = 16;
// column passes and pass C: FP64 lines with 10 elements per thread and at most 512
// threads (up to 256 VGPRs), FP32 lines with 8 and at most 1024
template <typename R> constexpr int gen_e() { return sizeof(R) == 8 ? 10 : 8; }
template <typename R> constexpr int gen_maxthr() { return sizeof(R) == 8 ? 512 : 1024; }
constexpr int kGenMaxStages = 24;
constexpr int kGenStageMax = 16;   // largest stage radix (any product of 2, 3 and 5 up to it)
// Largest stage radix of each mixed-radix kernel (a thread holds up to that many
// elements in a stage, beside what the kernel keeps across transforms: the spectrum in
// the symbol pass, sums and interpolation records in pass C), chosen so that none
// spills and a line of kGenMaxN points still fits the thread limit.
enum GenKernel { kGenRows = 0, kGenCols = 1, kGenSym = 2, kGenComb = 3 };
#ifndef HP_GEN_SMAX64
#define HP_GEN_SMAX64 12
#endif
template <typename R>
constexpr int gen_smax(int k) {
  return sizeof(R) == 8 ? (k == kGenRows || k == kGenCols ? kGenStageMax : HP_GEN_SMAX64) : (k == kGenRows ? 12 : 8);
}
// (pass A picks between kGenStageMax and kGenRowSmaxLo per length: gen_rows_smax)
constexpr int kGenMaxN = 4800;
struct GenPlan {
  int n, nst, nthr, tc;
  int smax;   // the stage-radix cap the plan was made for (selects the kernel)
  int radix[kGenMaxStages];
};
constexpr int kGenRowSmaxLo = 12;   // pass A's cap at three waves per SIMD
int gen_rows_smax(int real_kind, int n);
// Fills *gp for length n, E elements per thread and at most maxthr threads per
// line; false if n is not a product of 2, 3 and 5 within kGenMaxN or does not fit.
// order: radix schedule (0: the largest stage radix up to kGenStageMax that divides what
// is left, first — 2400 = 16 15 10; 1: the same stages ascending; 2: the same with the
// first moved last; 3: radices 4, 2, 3, 5 only, each as often as it divides what is
// left); nthr_req > 0 asks for that many threads per line (false if it does not fit E
// and maxthr).
bool make_gen_plan(int n, int E, int maxthr, GenPlan* gp, int order = 0, int nthr_req = 0,
                   int smax = kGenStageMax);
constexpr int kGenOrders = 4;
// Every mixed-radix kernel can take lines of length n.
bool gen_length_ok(int n);
inline bool is_pow2_len(int n) { return n > 0 && (n & (n - 1)) == 0; }
// Column passes (strided axes) take the LDS-resident mixed-radix kernels for
// lengths that are not powers of two, and for FP64 power-of-two lengths above
// 2048, whose register-tile column kernel would not fit in LDS.
bool cols_use_gen(int real_kind, int n);

// Run-time choices of a transform pass (0 = the built-in choice): threads per line,
// lines per workgroup (column passes) and radix schedule of the mixed-radix passes,
// node groups per column tile of the power-of-two symbol pass, node splits (1 or 4)
// of the power-of-two pass C.  Only the radix schedule and the node splits change
// results (rounding: the order of the node sum).
struct PassTune {
  int nthr = 0, tc = 0, order = 0, ng = 0;
};
// slot kinds of the candidates below: 0 pass A (rows forward), 1 column pass (B, A', M),
// 2 pass C (rows inverse + combine)
constexpr int kTuneRows = 0, kTuneCols = 1, kTuneCombine = 2;
// Valid choices for one pass over lines of length n (S lines across for column passes;
// mode 1 = the symbol pass, K node fields); writes at most max and returns the count.
int tune_candidates(int real_kind, int kind, int n, int S, int mode, int K, PassTune* out, int max);

// ---- launchers (all enqueue on `st`, return the launch status) ----

// Pass A: forward transform along the contiguous axis.
// in_kind: 0 = complex128 input, 1 = complex64 input.  real_kind: 0 = FP64, 1 = FP32.
// Pass launchers take an optional pair of timing events `tev` (tev[0], tev[1]): the
// pass's kernel is then launched with hipExtLaunchKernelGGL, which stores the
// kernel's own start and end times in them.
hipError_t launch_rows_fwd(int real_kind, int in_kind, int n, const void* in, void* out, int rows,
                           size_t in_rs, size_t out_rs, int nrhs, const void* tw, const int* skip,
                           const PassTune& tune, hipStream_t st, const hipEvent_t* tev = nullptr);

// Strided-axis transform over column tiles: element (o, p, c) at o*n*S + p*S + c.
// mode 0: plain transform (dir -1/+1) of nfields fields;
// mode 1: forward, then for every node: symbol multiply and inverse (pass B).
struct ColsArgs {
  int real_kind, n, dir, mode;
  const void* in;
  void* out;
  int S, outer, nfields, nrhs;
  size_t in_rs, out_rs, in_fs, out_fs;
  const void* tw;
  const int* skip;
  const double* lam_ax;
  const double* lam_in;
  const NodeConst* nodes;
  int K;
  double scale;
  const uint16_t* store_mask;   // mode 1: [K][T] bit s = axis-0 index j + T*s uses node n
  int store_mask_thr;           // mixed-radix lengths: the T store_mask was built for (0: none)
  const uint8_t* slab_need;     // mode 0 over node fields: [K][outer] != 0 if the slab uses node n
  const uint8_t* store_need;    // mode 1, mixed-radix lengths: [K][n] != 0 if axis-0 index p uses node n
  PassTune tune;
  const hipEvent_t* tev = nullptr;   // timing events of the launch (see launch_rows_fwd)
};
hipError_t launch_cols(const ColsArgs& a, hipStream_t st);

// Pass C: inverse transform along the contiguous axis of the K node fields and
// the interpolation combine.  out_kind: 0 = complex128, 1 = complex64.
struct CombineArgs {
  int real_kind, out_kind, accumulate, n;
  const void* fields;
  size_t fs, frs;
  const double* pos;
  const uint64_t* grpmask;   // per workgroup: nodes used by any of its rows
  const uint64_t* rowmask;   // per row: nodes used by the row
  void* out;
  size_t out_rs;
  int rows, K, M, Mt, mo, nrhs;
  const void* tw;
  const int* skip;
  int order;           // real-axis interpolation degree in effect (1 = piecewise linear)
  const double* lag;   // order >= 2: real nodes [0, kMaxNodes), then for node n and stencil
                       // start n - r the inverse Lagrange denominator at kMaxNodes + 4n + r
  const double* posa;  // Ma >= 2: per point, the position among the damping nodes (bilinear in (c, a))
  int Ma;              // damping nodes of the bivariate scheme (0: univariate)
  PassTune tune;
  const hipEvent_t* tev = nullptr;   // timing events of the launch (see launch_rows_fwd)
};
constexpr int kLagTable = kMaxNodes * 5;
hipError_t launch_combine(const CombineArgs& a, hipStream_t st);
int combine_group_rows(int real_kind, int n);        // rows per workgroup of pass C
int symbol_pass_line_threads(int real_kind, int n);  // threads per line T of pass B
// threads per line of the built-in mixed-radix symbol-pass plan (0 if n has none) and
// the elements each thread holds
int gen_symbol_line_threads(int real_kind, int n);
int gen_symbol_elems(int real_kind);

// Stencil.  kind: 0 = FP64 (c128 -> c128), 1 = FP32 arithmetic c64 -> c64,
// 2 = FP32 arithmetic c64 -> c128, 3 = FP64 residual y = f - P u (c128).
struct StencilArgs {
  int kind, dim;
  int n[3];
  double ih2[3];
  const void* u;
  void* y;
  const void* coef;
  const void* f;     // residual mode: right-hand side, same strides as u
  size_t u_rs, y_rs;
  int nrhs;
  const int* skip;
};
hipError_t launch_stencil(const StencilArgs& a, hipStream_t st);

// Krylov kernels (FP64).  Basis of one right-hand side: (restart + 1) vectors of
// npts points; bases of consecutive right-hand sides are vrs elements apart.
struct KrylovArgs {
  cpx<double>* V;
  size_t npts, vrs;
  KState* state;
  cpx<double>* part;
  int* skip_step;   // 1 when the current cycle's Arnoldi process has ended
  int* done;        // 1 when the right-hand side has converged
  int* host_stop;   // pinned host copy of skip_step written by the kernels (may be null)
  int* host_done;   // pinned host copy of done written by the kernels (may be null)
  int nrhs, restart;
};
// ||f|| of f [nrhs][npts] (stride frs) -> state.fnorm, target; done/skip_step for f = 0.
hipError_t launch_fnorm(const KrylovArgs& a, const cpx<double>* f, size_t frs, double rtol, hipStream_t st);
// ||v_0|| (v_0 holds the true residual) -> beta, convergence test, cycle reset.
hipError_t launch_cycle_start(const KrylovArgs& a, double rtol, hipStream_t st);
hipError_t launch_scale_v0(const KrylovArgs& a, hipStream_t st);
// Arnoldi step j (slot j holds u_j, slot j+1 holds w = A u_j): the one reduction
// of the step (partial sums, then one block per right-hand side finishes it).
hipError_t launch_arnoldi_dots(const KrylovArgs& a, int j, hipStream_t st);
// The same with w = P_N z computed by the sweep from s (s.u = z, kinds 0 and 2 of the
// stencil, not the residual form) and stored in slot j+1.
hipError_t launch_arnoldi_dots_stencil(const KrylovArgs& a, int j, const StencilArgs& s, hipStream_t st);
// Arnoldi step j: slot j <- v_j, slot j+1 <- u_{j+1}.
hipError_t launch_arnoldi_update(const KrylovArgs& a, int j, hipStream_t st);
// The same for FP64 2-D grids with rows of 512, 1024 or 2048 points (update_rows_fits),
// which also writes the row transform of u_{j+1} into t ([nrhs][npts]), pass A of
// the next step's apply.
bool update_rows_fits(int real_kind, int dim, int n_last);
hipError_t launch_arnoldi_update_rows(const KrylovArgs& a, int j, void* t, int n_last, const void* tw,
                                      hipStream_t st);
hipError_t launch_backsolve(const KrylovArgs& a, hipStream_t st);
// ||w||^2 of each right-hand side into KState::fnorm_plain (which = 0) or, divided
// by it, into KState::relres_plain (which = 1); all right-hand sides.
hipError_t launch_plain_norm(const KrylovArgs& a, const cpx<double>* w, size_t wrs, int which, hipStream_t st);
hipError_t launch_lincomb(const KrylovArgs& a, cpx<double>* out, size_t out_rs, bool accumulate, hipStream_t st);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);
// ---- grouped Arnoldi steps (several solver sessions, any mix of the grids below,
// one launch per pass) ----
constexpr int kMaxGroup = 8;
// One right-hand side of a right-preconditioned session whose preconditioner runs in
// FP32 (mixed precision): its plan's tables and its buffers for the current step j.
struct GroupMember {
  int dim, n[3];
  size_t npts;
  int K, M, Mt, mo, order, Ma;
  int interp;                 // InterpMode of the combine
  double scale;               // 1 / npts
  const void* tw[3];          // FP32 twiddles per axis
  const double* lam_ax;
  const double* lam_in;
  const NodeConst* nodes;
  const uint16_t* store_mask;
  const uint8_t* slab_need;
  const double* pos;
  const double* posa;
  const uint64_t* grpmask;
  const uint64_t* rowmask;
  const double* lag;
  const void* coef32;         // stencil coefficients {gamma^2, beta} in FP32
  double ih2[3];
  void* t;                    // pass A output
  void* fields;               // node fields
  void* z;                    // Q u_j (complex64)
  cpx<double>* V;             // the member's basis
  KState* state;
  cpx<double>* part;
  int* skip_step;
  int* host_stop;
  int j, restart;
  int ng_b;                   // node groups of the symbol pass (0: the single-plan choice)
};
// Whether a member's grid and options are ones the grouped kernels take (the grouped
// step then gives bitwise the result of the member's own step).
bool group_member_ok(const GroupMember& m);
// Arnoldi step of every member (count <= kMaxGroup): passes A (A'), B, (M), C, the
// dot-product sweep with the stencil, the finishing kernel and the update, one
// launch each over all members.
hipError_t launch_group_step(const GroupMember* m, int count, hipStream_t st);
// Device address of this device's copy of the static apply workspace
// (HP_STATIC_SCRATCH_BYTES), looked up once per device, on the current device.
hipError_t static_scratch(void** out);
hipError_t launch_rsub(const cpx<double>* b, size_t b_rs, cpx<double>* v, size_t v_rs, size_t n, int nrhs,
                       const int* skip, hipStream_t st);

// ---- plan set-up on the device (FP64) ----
struct MediaScan {
  double cmin, cmax, zmax, a0;
  int bad;          // non-finite or out-of-range value
  int layer_bad;    // zeta > 0 where |c - c0| > 1e-12 c0
  int a_varies;     // a is not uniform
  int pad;
};
constexpr int kScanBlocks = 256;
// per-block partial scans of the media (a, zeta may be null)
hipError_t launch_media_scan(const double* c, const double* a, const double* zeta, size_t n, double c0,
                             MediaScan* partial, hipStream_t st);

struct NodeTable {
  int M, Mt, mo, has_layer;
  int order;   // real-axis interpolation degree in effect (1 = piecewise linear, else Lagrange)
  int Ma;      // second-axis nodes of a tensor scheme, node (m, r) = m + M r (0: off)
  int second;  // the second axis: 0 damping a (bivariate), 1 Im gamma = -c zeta (layer tensor)
  double cnode[kMaxNodes];
  double znode[kMaxNodes + 1];
  double anode[kMaxNodes];
};
// per point: interpolation record (see decode_pos) and stencil coefficients
// {gamma^2, omega^2 + i omega a - 2 gamma^2 sum_j h_j^-2} in FP64 (and FP32 if coef32)
// (and, for the bivariate scheme, the damping position posa)
hipError_t launch_plan_points(const double* c, const double* a, const double* zeta, size_t n, const NodeTable& T,
                              double omega, double sum_ih2, double* pos, double* posa, cpx<double>* coef64,
                              cpx<float>* coef32, hipStream_t st);
// per row of nl points: bit k set if some point of the row has a non-zero weight on node k
hipError_t launch_row_masks(const double* pos, const double* posa, int nl, size_t rows, const NodeTable& T,
                            uint64_t* rowmask, hipStream_t st);

}  // namespace hp
