// Host side of the library: plan set-up in FP64 (node placement, per-point
// interpolation records, stencil coefficients, symbol and twiddle tables), the
// enqueue sequences of apply and matvec, and the restarted-GMRES driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/helmpre.h"
#include "hp_internal.h"

using hp::cpx;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t alloc(size_t b) {
    release();
    if (b == 0) return hipSuccess;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) { p = nullptr; return e; }
    bytes = b;
    return hipSuccess;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

}  // namespace

struct hp_plan_s;
namespace {
void load_tune(hp_plan_s& P);
void save_tune(const hp_plan_s& P);

// Arnoldi steps of small grids run as captured HIP graphs when HP_STEP_GRAPHS=1 (off
// by default: on this runtime a graph launch of a step costs more than its seven
// direct launches, 256^2 FP64 solve 5.5 -> 6.1 ms).
bool step_graphs_enabled() {
  const char* v = std::getenv("HP_STEP_GRAPHS");
  return v && v[0] == '1';
}
}  // namespace

struct hp_plan_s {
  int dim = 2;
  int n[3] = {1, 1, 1};
  double len[3] = {1, 1, 1};
  size_t npts = 0;
  double omega = 0;
  int prec = HP_FP64;
  int symbol = HP_SYMBOL_CONTINUOUS;
  int max_nrhs = 1;
  // nodes
  int K = 1, M = 1, Mt = 0, mo = 0;
  double cmin = 0, cmax = 0, zmax = 0;
  double cnode[64] = {0}, znode[65] = {0}, ahat[64] = {0}, gre[64] = {0}, gim[64] = {0};
  // device data
  DevBuf nodes, pos, grpmask, rowmask, slabneed, storemask, coef64, coef32, lam_ax, lam_in, tw64[3], tw32[3];
  int order = 1;   // real-axis interpolation degree in effect
  DevBuf lagtab;   // Lagrange table of CombineArgs::lag (order >= 2)
  hp::PassTune tune[5];   // run-time choices of passes A, A', B, M, C (hp_plan_autotune)
  int tune_gen = 0;        // bumped when they change (captured step graphs become stale)
  int Ma = 0;      // second-axis nodes of a tensor scheme: damping (c, a) or Im gamma (layer tensor)
  int tensor = 0;  // 1: layer tensor (second axis Im gamma)
  double anode[64] = {0};
  DevBuf posa;     // per point: position among the damping nodes (Ma >= 2)
  // node usage counts for the byte model of the passes
  double rows_used = 0;    // sum over pass-C rows of the nodes the row uses
  double slabs_used = 0;   // sum over nodes of the axis-0 indices that use the node
  int smask_thr = 0;       // mixed-radix lengths: threads per line storemask was built for
  DevBuf t, fields;                  // apply workspace
  // Who last wrote t, in enqueue order: a solver session whose fused Arnoldi update
  // left the row transform of its u_{t_step} there, or nobody (an apply overwrote it).
  const void* t_owner = nullptr;
  int t_step = -1;
  // solver workspace of hp_solve (sessions created with hp_solver_create own theirs)
  struct SolverWs* solver_ws_ptr = nullptr;
  int arnoldi_k = -1;   // basis vectors the last hp_arnoldi left in that workspace (-1: none)
  struct SolverWs* inner_ws_ptr = nullptr;   // the inner solves of hp_arnoldi's inverse operators
  // pass timer (hp_plan_time_pass): the start and end times of every launch of one pass
  int timer_slot = -1;
  size_t timer_n = 0;                 // launches recorded since the last read
  std::vector<hipEvent_t> timer_ev;   // 2 per launch, created on demand and reused

  int real_kind() const { return prec == HP_FP64 ? 0 : 1; }
  size_t fsize() const { return prec == HP_FP64 ? 16 : 8; }
  const void* tw(int axis) const { return prec == HP_FP64 ? tw64[axis].p : tw32[axis].p; }
  void release_all() {
    for (DevBuf* b : {&nodes, &pos, &grpmask, &rowmask, &slabneed, &storemask, &coef64, &coef32, &lam_ax, &lam_in, &t,
                      &fields, &lagtab, &posa})
      b->release();
    for (int i = 0; i < 3; ++i) { tw64[i].release(); tw32[i].release(); }
    release_solver_ws();
    for (hipEvent_t e : timer_ev) (void)hipEventDestroy(e);
    timer_ev.clear();
    timer_n = 0;
  }
  void release_solver_ws();
};

namespace {

thread_local char g_last_error[256] = "";

hp_status record(hipError_t e, const char* where, int line) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s (line %d): %s", where, line, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? HP_E_NOMEM : HP_E_DEVICE;
}

#define from_hip(e) ((e) == hipSuccess ? HP_OK : record((e), __func__, __LINE__))

#define HP_TRY(expr)                         \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return from_hip(e_); \
  } while (0)

// Real interpolation nodes (Section 4.1); with an absorbing layer the
// background speed c0 must be one of them (Section 4.4).  Reading: two
// equidistant runs on [cmin, c0] and [c0, cmax]; the number of intervals below
// c0 is the nearest integer (ties downwards) to (c0-cmin)/(cmax-cmin)*(M-1),
// kept in [1, M-2] when c0 is strictly inside (M raised to 3 if smaller).
hp_status place_real_nodes(hp_plan_s& P, const hp_plan_opts& o, double c0, bool layer) {
  int M = o.m_real;
  if (M < 1 || M > hp::kMaxNodes) return HP_E_INVALID;
  if (o.nodes_real) {
    for (int i = 0; i < M; ++i) {
      double v = o.nodes_real[i];
      if (!(v > 0) || !std::isfinite(v) || (i && !(v > o.nodes_real[i - 1]))) return HP_E_INVALID;
      P.cnode[i] = v;
    }
    P.M = M;
    P.mo = -1;
    for (int i = 0; i < M; ++i)
      if (P.cnode[i] == c0) P.mo = i;
    if (layer && P.mo < 0) return HP_E_LAYER;
    if (P.mo < 0) P.mo = 0;
    return HP_OK;
  }
  if (M == 1) {                        // one-node preconditioner Q_1 at c0
    P.M = 1;
    P.cnode[0] = c0;
    P.mo = 0;
    return HP_OK;
  }
  const double lo = P.cmin, hi = P.cmax;
  if (!(hi > lo)) {                    // homogeneous medium: a single node
    if (layer && lo != c0) return HP_E_LAYER;
    P.M = 1;
    P.cnode[0] = lo;
    P.mo = 0;
    return HP_OK;
  }
  if (!layer) {
    const double step = (hi - lo) / (M - 1);
    for (int i = 0; i < M; ++i) P.cnode[i] = lo + step * i;
    P.cnode[M - 1] = hi;
    P.M = M;
    P.mo = 0;
    return HP_OK;
  }
  if (c0 < lo || c0 > hi) return HP_E_LAYER;
  int below;
  if (c0 == lo) {
    below = 0;
  } else if (c0 == hi) {
    below = M - 1;
  } else {
    M = std::max(M, 3);
    const double r = (c0 - lo) / (hi - lo) * (M - 1);
    below = (int)std::ceil(r - 0.5);
    below = std::min(std::max(below, 1), M - 2);
  }
  for (int i = 0; i < M; ++i) {
    if (i < below) P.cnode[i] = lo + (c0 - lo) * ((double)i / below);
    else if (i == below) P.cnode[i] = c0;
    else P.cnode[i] = c0 + (hi - c0) * ((double)(i - below) / (M - 1 - below));
  }
  if (below != M - 1) P.cnode[M - 1] = hi;
  P.M = M;
  P.mo = below;
  return HP_OK;
}

// Interpolation record of a point (see decode_pos in the kernels).
double encode_point(const hp_plan_s& P, double c, double z) {
  if (P.Mt > 0 && z > 0.0) {
    double zz = std::min(z, P.znode[P.Mt]);
    int j = (int)(std::upper_bound(P.znode, P.znode + P.Mt + 1, zz) - P.znode) - 1;
    j = std::min(std::max(j, 0), P.Mt - 1);
    const double t = (zz - P.znode[j]) / (P.znode[j + 1] - P.znode[j]);
    return -(1.0 + j + t);
  }
  if (P.M == 1) return 0.0;
  double cc = std::min(std::max(c, P.cnode[0]), P.cnode[P.M - 1]);
  int s = (int)(std::upper_bound(P.cnode, P.cnode + P.M, cc) - P.cnode) - 1;
  s = std::min(std::max(s, 0), P.M - 2);
  const double t = (cc - P.cnode[s]) / (P.cnode[s + 1] - P.cnode[s]);
  return s + t;
}

void point_nodes(const hp_plan_s& P, double pos, int& A, int& B, double& t) {
  if (pos >= 0) {
    if (P.M == 1) { A = B = 0; t = 0; return; }
    int s = std::min((int)pos, P.M - 2);
    A = s; B = s + 1; t = pos - s;
  } else {
    double q = -pos - 1.0;
    int s = std::min((int)q, P.Mt - 1);
    A = s == 0 ? P.mo : P.M + s - 1; B = P.M + s; t = q - s;
  }
}

double lambda_1d(int k, int n, double len, int symbol) {
  if (symbol == HP_SYMBOL_CONTINUOUS) {
    const int ks = k < n / 2 ? k : k - n;
    const double xi = 2.0 * M_PI * ks / len;
    return xi * xi;
  }
  const double h = len / n;
  const double s = std::sin(M_PI * k / n);
  return 4.0 / (h * h) * s * s;
}

template <typename T>
hipError_t upload(DevBuf& b, const std::vector<T>& v) {
  hipError_t e = b.alloc(v.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

hp_status check_grid(const hp_grid* g, int prec) {
  if (!g || (g->dim != 2 && g->dim != 3)) return HP_E_SHAPE;
  const int hi = prec == HP_FP64 ? 2048 : 4096;
  for (int d = 0; d < g->dim; ++d) {
    // powers of two, or even products of 2, 3 and 5 (mixed-radix lines held in LDS)
    const int n = g->n[d];
    const bool ok = pow2_in(n, 8, hi) || (n >= 8 && n % 2 == 0 && hp::gen_length_ok(n));
    if (!ok) return HP_E_SHAPE;
    if (!(g->len[d] > 0) || !std::isfinite(g->len[d])) return HP_E_INVALID;
  }
  // point indices are 32-bit in the kernels
  size_t np = 1;
  for (int d = 0; d < g->dim; ++d) np *= (size_t)g->n[d];
  if (np >= ((size_t)1 << 32)) return HP_E_SHAPE;
  return HP_OK;
}

}  // namespace

extern "C" {

const char* hp_last_error(void) { return g_last_error; }

const char* hp_status_str(hp_status st) {
  switch (st) {
    case HP_OK: return "ok";
    case HP_E_INVALID: return "invalid argument";
    case HP_E_SHAPE: return "unsupported grid shape";
    case HP_E_MEDIA: return "invalid media or vanishing symbol denominator";
    case HP_E_LAYER: return "wave speed differs from c0 inside the absorbing layer";
    case HP_E_NONFINITE: return "non-finite input";
    case HP_E_DEVICE: return "HIP device error";
    case HP_E_NOMEM: return "out of device memory";
    case HP_E_NOT_CONVERGED: return "not converged";
  }
  return "unknown status";
}

size_t hp_plan_workspace_bytes(const hp_grid* g, const hp_plan_opts* o, int K) {
  if (!g || !o) return 0;
  size_t npts = 1;
  for (int d = 0; d < g->dim; ++d) npts *= (size_t)g->n[d];
  const size_t fs = o->precision == HP_FP64 ? 16 : 8;
  const size_t nr = (size_t)std::max(1, o->max_nrhs);
  size_t b = nr * npts * fs * (size_t)(K + 1);      // t and the K node fields
  b += npts * (8 + 32 + (o->precision == HP_FP64 ? 0 : 16));   // pos, coef64, coef32
  if (o->m_damp >= 2 || o->layer_tensor) b += npts * 8;       // posa
  return b;
}

size_t hp_solve_workspace_bytes(const hp_grid* g, int restart, int nrhs) {
  if (!g) return 0;
  size_t npts = 1;
  for (int d = 0; d < g->dim; ++d) npts *= (size_t)g->n[d];
  const size_t nr = (size_t)std::max(1, nrhs);
  return nr * (npts * 16 * (size_t)(restart + 3) + sizeof(hp::KState) +
               (size_t)hp::kRedBlocks * hp::kPartSlots * 16 + 16);
}

hp_status hp_plan_create(hp_plan* out, const hp_grid* grid, double omega, const double* c, const double* a,
                         const hp_layer* layer, const hp_plan_opts* opts, void* stream) {
  if (!out) return HP_E_INVALID;
  *out = nullptr;
  if (!opts || !c) return HP_E_INVALID;
  if (opts->precision != HP_FP64 && opts->precision != HP_MIXED) return HP_E_INVALID;
  if (opts->symbol != HP_SYMBOL_CONTINUOUS && opts->symbol != HP_SYMBOL_DISCRETE) return HP_E_INVALID;
  if (opts->max_nrhs < 1 || opts->max_nrhs > 4096) return HP_E_INVALID;
  if (!(omega > 0) || !std::isfinite(omega)) return HP_E_INVALID;
  if (!(opts->a_floor >= 0) || !std::isfinite(opts->a_floor)) return HP_E_INVALID;
  hp_status st = check_grid(grid, opts->precision);
  if (st) return st;
  const double c0 = layer ? layer->c0 : 1.0;
  if (!(c0 > 0) || !std::isfinite(c0)) return HP_E_INVALID;

  hp_plan_s* P = new (std::nothrow) hp_plan_s();
  if (!P) return HP_E_NOMEM;
  auto fail = [&](hp_status s) {
    P->release_all();
    delete P;
    return s;
  };
  P->dim = grid->dim;
  P->npts = 1;
  for (int d = 0; d < grid->dim; ++d) {
    P->n[d] = grid->n[d];
    P->len[d] = grid->len[d];
    P->npts *= (size_t)grid->n[d];
  }
  P->omega = omega;
  P->prec = opts->precision;
  P->symbol = opts->symbol;
  P->max_nrhs = opts->max_nrhs;
  const size_t np = P->npts;
  const double* zeta = layer ? layer->zeta : nullptr;

  hipStream_t hs = (hipStream_t)stream;
  hipError_t e;
  // The raw media go to the device once; the per-point set-up runs there.
  DevBuf dc, da, dz, dscan;
  if ((e = dc.alloc(np * 8)) != hipSuccess) return fail(from_hip(e));
  if ((e = hipMemcpyAsync(dc.p, c, np * 8, hipMemcpyHostToDevice, hs)) != hipSuccess) return fail(from_hip(e));
  if (a) {
    if ((e = da.alloc(np * 8)) != hipSuccess) return fail(from_hip(e));
    if ((e = hipMemcpyAsync(da.p, a, np * 8, hipMemcpyHostToDevice, hs)) != hipSuccess) return fail(from_hip(e));
  }
  if (zeta) {
    if ((e = dz.alloc(np * 8)) != hipSuccess) return fail(from_hip(e));
    if ((e = hipMemcpyAsync(dz.p, zeta, np * 8, hipMemcpyHostToDevice, hs)) != hipSuccess) return fail(from_hip(e));
  }
  auto cleanup = [&]() { dc.release(); da.release(); dz.release(); dscan.release(); };
  auto failc = [&](hp_status s) { cleanup(); return fail(s); };

  // media checks and ranges
  if ((e = dscan.alloc(sizeof(hp::MediaScan) * hp::kScanBlocks)) != hipSuccess) return failc(from_hip(e));
  if ((e = hp::launch_media_scan((const double*)dc.p, (const double*)da.p, (const double*)dz.p, np, c0,
                                 (hp::MediaScan*)dscan.p, hs)) != hipSuccess)
    return failc(from_hip(e));
  std::vector<hp::MediaScan> scan(hp::kScanBlocks);
  if ((e = hipMemcpyAsync(scan.data(), dscan.p, sizeof(hp::MediaScan) * hp::kScanBlocks, hipMemcpyDeviceToHost, hs)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(hs)) != hipSuccess)
    return failc(from_hip(e));
  P->cmin = INFINITY;
  P->cmax = -INFINITY;
  P->zmax = 0;
  bool bad = false, layer_bad = false, a_varies = false;
  for (const hp::MediaScan& m : scan) {
    P->cmin = std::min(P->cmin, m.cmin);
    P->cmax = std::max(P->cmax, m.cmax);
    P->zmax = std::max(P->zmax, m.zmax);
    bad = bad || m.bad;
    layer_bad = layer_bad || m.layer_bad;
    a_varies = a_varies || m.a_varies;
  }
  if (bad) return failc(HP_E_MEDIA);
  const bool q1 = opts->m_real == 1 && !opts->nodes_real;
  const bool has_layer = P->zmax > 0 && !q1;
  // layer tensor: speed nodes on [c_min, c_max] by Im gamma nodes on [-max(c zeta), 0]
  // (c need not equal c0 in the layer); the layer legs are replaced
  const bool tensor = has_layer && opts->layer_tensor;
  if (tensor && (opts->m_damp >= 2 || opts->interp_order >= 2 || opts->m_layer < 1 ||
                 opts->m_layer + 1 > hp::kMaxNodes))
    return failc(HP_E_INVALID);
  st = place_real_nodes(*P, *opts, c0, has_layer && !tensor);
  if (st) return failc(st);
  P->Mt = 0;
  if (tensor) {
    double gmax = 0.0;
    for (size_t i = 0; i < np; ++i) gmax = std::max(gmax, c[i] * zeta[i]);
    P->tensor = 1;
    P->Ma = opts->m_layer + 1;
    for (int r = 0; r < P->Ma; ++r) P->anode[r] = -gmax + gmax * ((double)r / (P->Ma - 1));
    P->anode[P->Ma - 1] = 0.0;
    if (P->M * P->Ma > hp::kMaxNodes) return failc(HP_E_INVALID);
  } else if (has_layer) {
    const int Mt = opts->m_layer;
    if (Mt < 1 || P->M + Mt > hp::kMaxNodes) return failc(HP_E_INVALID);
    P->znode[0] = 0;
    for (int j = 1; j <= Mt; ++j) {
      if (opts->nodes_zeta) {
        P->znode[j] = opts->nodes_zeta[j - 1];
        if (!(P->znode[j] > P->znode[j - 1]) || !std::isfinite(P->znode[j])) return failc(HP_E_INVALID);
      } else {
        P->znode[j] = (j == Mt) ? P->zmax : P->zmax * ((double)j / Mt);
      }
    }
    P->Mt = Mt;
    if (layer_bad) return failc(HP_E_LAYER);
  }
  P->K = P->tensor ? P->M * P->Ma : P->M + P->Mt;
  // real-axis interpolation: piecewise linear (Section 4.1), or piecewise Lagrange of
  // degree 2 or 3 on consecutive nodes (at most M - 1)
  if (opts->interp_order < 0 || opts->interp_order > 3) return failc(HP_E_INVALID);
  P->order = std::max(1, std::min(opts->interp_order, P->M - 1));
  // bivariate (c, a): equidistant damping nodes on [a_min, a_max], real node (c_m, a_r)
  // = node m + M r; no layer (its nodes would need a third axis), piecewise linear
  if (opts->m_damp < 0 || opts->m_damp > hp::kMaxNodes) return failc(HP_E_INVALID);
  if (opts->m_damp >= 2) {
    if (has_layer || opts->interp_order >= 2 || opts->a_nodes || opts->layer_tensor) return failc(HP_E_INVALID);
    double amin = a ? a[0] : 0.0, amax = amin;
    if (a)
      for (size_t i = 1; i < np; ++i) { amin = std::min(amin, a[i]); amax = std::max(amax, a[i]); }
    if (amax > amin) {
      P->Ma = opts->m_damp;
      if (P->M * P->Ma > hp::kMaxNodes) return failc(HP_E_INVALID);
      for (int r = 0; r < P->Ma; ++r) P->anode[r] = amin + (amax - amin) * ((double)r / (P->Ma - 1));
      P->anode[P->Ma - 1] = amax;
      P->K = P->M * P->Ma;
    }
  }
  hp::NodeTable T{};
  T.M = P->M;
  T.Mt = P->Mt;
  T.mo = P->mo;
  T.has_layer = has_layer && !tensor ? 1 : 0;
  T.second = tensor ? 1 : 0;
  T.order = P->order;
  T.Ma = P->Ma;
  for (int i = 0; i < P->Ma; ++i) T.anode[i] = P->anode[i];
  for (int i = 0; i < P->M; ++i) T.cnode[i] = P->cnode[i];
  for (int i = 0; i <= P->Mt; ++i) T.znode[i] = P->znode[i];
  {
    // node positions, then 1 / prod_{k != n} (c_n - c_k) over the stencil starting at n - r
    std::vector<double> lag(hp::kLagTable, 0.0);
    for (int i = 0; i < P->M; ++i) lag[i] = P->cnode[i];
    if (P->order >= 2) {
      for (int nn = 0; nn < P->M; ++nn)
        for (int r = 0; r <= P->order; ++r) {
          const int a = nn - r;
          if (a < 0 || a > P->M - 1 - P->order) continue;
          double den = 1.0;
          for (int k = a; k <= a + P->order; ++k)
            if (k != nn) den *= P->cnode[nn] - P->cnode[k];
          lag[hp::kMaxNodes + 4 * nn + r] = 1.0 / den;
        }
    }
    if ((e = upload(P->lagtab, lag)) != hipSuccess) return failc(from_hip(e));
  }

  // per-point records and stencil coefficients {gamma^2, beta} (Section 5 with
  // the complex speed of Section 4.4), in FP64 on the device
  double sih2 = 0;
  for (int d = 0; d < P->dim; ++d) {
    const double h = P->len[d] / P->n[d];
    sih2 += 1.0 / (h * h);
  }
  if ((e = P->pos.alloc(np * 8)) != hipSuccess) return failc(from_hip(e));
  if (P->Ma >= 2 && (e = P->posa.alloc(np * 8)) != hipSuccess) return failc(from_hip(e));
  if ((e = P->coef64.alloc(np * 32)) != hipSuccess) return failc(from_hip(e));
  if (P->prec == HP_MIXED && (e = P->coef32.alloc(np * 16)) != hipSuccess) return failc(from_hip(e));
  if ((e = hp::launch_plan_points((const double*)dc.p, (const double*)da.p, (const double*)dz.p, np, T, omega, sih2,
                                  (double*)P->pos.p, (double*)P->posa.p, (cpx<double>*)P->coef64.p,
                                  (cpx<float>*)P->coef32.p, hs)) != hipSuccess)
    return failc(from_hip(e));

  // Node usage.  Each point has at most two non-zero weights, so a row of
  // pass C only needs the node fields its points use; the passes before it
  // neither write nor transform the rest.
  const int nl = P->n[P->dim - 1];
  const size_t rows = np / nl;
  if ((e = P->rowmask.alloc(rows * 8)) != hipSuccess) return failc(from_hip(e));
  if ((e = hp::launch_row_masks((const double*)P->pos.p, (const double*)P->posa.p, nl, rows, T,
                                (uint64_t*)P->rowmask.p, hs)) != hipSuccess)
    return failc(from_hip(e));
  std::vector<uint64_t> rm(rows, 0);
  if ((e = hipMemcpyAsync(rm.data(), P->rowmask.p, rows * 8, hipMemcpyDeviceToHost, hs)) != hipSuccess ||
      (e = hipStreamSynchronize(hs)) != hipSuccess)
    return failc(from_hip(e));

  // symbol damping per node: uniform a as is, a(c_m) if given, otherwise the
  // weight-averaged a over the points each real node serves; layer nodes take
  // the damping of c_o.  The floor applies at the end to the nodes of real speed.
  const double a0 = a ? a[0] : 0.0;
  for (int m = 0; m < P->M; ++m) P->ahat[m] = a0;
  if (opts->a_nodes) {
    for (int m = 0; m < P->M; ++m) {
      if (!(opts->a_nodes[m] >= 0) || !std::isfinite(opts->a_nodes[m])) return failc(HP_E_INVALID);
      P->ahat[m] = opts->a_nodes[m];
    }
  } else if (a_varies && (P->Ma < 2 || P->tensor)) {
    std::vector<double> num(P->K, 0.0), den(P->K, 0.0);
    double mean = 0;
    for (size_t i = 0; i < np; ++i) {
      int A, B;
      double t;
      point_nodes(*P, encode_point(*P, c[i], has_layer ? zeta[i] : 0.0), A, B, t);
      auto add = [&](int n, double w) {
        if (n < P->M) { num[n] += w * a[i]; den[n] += w; }
      };
      if (A == B) add(A, 1.0);
      else { add(A, 1.0 - t); add(B, t); }
      mean += a[i];
    }
    mean /= (double)np;
    for (int m = 0; m < P->M; ++m) P->ahat[m] = den[m] > 0 ? num[m] / den[m] : mean;
  }
  for (int m = 0; m < P->M; ++m) { P->gre[m] = P->cnode[m]; P->gim[m] = 0; }
  if (P->tensor) {   // layer tensor: node m + M r carries gamma = c_m + i g_r and the damping of c_m
    for (int r = P->Ma - 1; r >= 0; --r)
      for (int m = 0; m < P->M; ++m) {
        P->gre[m + P->M * r] = P->cnode[m];
        P->gim[m + P->M * r] = P->anode[r];
        P->ahat[m + P->M * r] = P->ahat[m];
      }
  } else {
    for (int r = 0; r < P->Ma; ++r)   // bivariate: node m + M r carries (c_m, a_r)
      for (int m = 0; m < P->M; ++m) {
        P->gre[m + P->M * r] = P->cnode[m];
        P->gim[m + P->M * r] = 0;
        P->ahat[m + P->M * r] = P->anode[r];
      }
  }
  for (int j = 1; j <= P->Mt; ++j) {
    P->ahat[P->M + j - 1] = P->ahat[P->mo];
    P->gre[P->M + j - 1] = c0;
    P->gim[P->M + j - 1] = -c0 * P->znode[j];
  }
  // Floor (the standing assumption a_min > 0 of Section 3 where a = 0): only
  // nodes of real speed can have a vanishing symbol denominator, at |xi| =
  // omega / c_n; a node with Im gamma_n < 0 keeps its damping.
  for (int k = 0; k < P->K; ++k)
    if (P->gim[k] == 0.0) P->ahat[k] = std::max(P->ahat[k], opts->a_floor);

  // symbol constants and tables
  std::vector<hp::NodeConst> nc(P->K);
  for (int k = 0; k < P->K; ++k) {
    const double gr = P->gre[k], gi = P->gim[k];
    nc[k] = {omega * omega, omega * P->ahat[k], gr * gr - gi * gi, 2 * gr * gi};
  }
  std::vector<double> lam0(P->n[0]);
  for (int k = 0; k < P->n[0]; ++k) lam0[k] = lambda_1d(k, P->n[0], P->len[0], P->symbol);
  size_t S = np / P->n[0];
  std::vector<double> lamin(S);
  if (P->dim == 2) {
    for (int k = 0; k < P->n[1]; ++k) lamin[k] = lambda_1d(k, P->n[1], P->len[1], P->symbol);
  } else {
    std::vector<double> l1(P->n[1]), l2(P->n[2]);
    for (int k = 0; k < P->n[1]; ++k) l1[k] = lambda_1d(k, P->n[1], P->len[1], P->symbol);
    for (int k = 0; k < P->n[2]; ++k) l2[k] = lambda_1d(k, P->n[2], P->len[2], P->symbol);
    for (int k1 = 0; k1 < P->n[1]; ++k1)
      for (int k2 = 0; k2 < P->n[2]; ++k2) lamin[(size_t)k1 * P->n[2] + k2] = l1[k1] + l2[k2];
  }
  // a vanishing denominator is only possible for a real node without damping
  for (int k = 0; k < P->K; ++k) {
    if (nc[k].aim != 0.0 || nc[k].gim != 0.0) continue;
    for (int k0 = 0; k0 < P->n[0]; ++k0)
      for (size_t ci = 0; ci < S; ++ci)
        if (nc[k].are - nc[k].gre * (lam0[k0] + lamin[ci]) == 0.0) return failc(HP_E_MEDIA);
  }

  const int G = hp::combine_group_rows(P->real_kind(), nl);
  std::vector<uint64_t> gm((rows + G - 1) / G, 0);
  for (size_t r = 0; r < rows; ++r) {
    gm[r / G] |= rm[r];
    P->rows_used += (double)__builtin_popcountll(rm[r]);
  }
  const int n0 = P->n[0];
  const size_t rows_per_slab = rows / n0;
  std::vector<uint8_t> need((size_t)P->K * n0, 0);
  for (int i0 = 0; i0 < n0; ++i0) {
    uint64_t m = 0;
    for (size_t r = 0; r < rows_per_slab; ++r) m |= rm[(size_t)i0 * rows_per_slab + r];
    for (int k = 0; k < P->K; ++k)
      if ((m >> k) & 1ull) { need[(size_t)k * n0 + i0] = 1; P->slabs_used += 1.0; }
  }
  // store masks of the symbol pass: bit e of thread j = axis-0 index j + Tb*e (for
  // mixed-radix lengths, with the built-in plan's Tb; a tuned plan with another
  // thread count reads `need` directly)
  std::vector<uint16_t> smask(1, 0);
  P->smask_thr = 0;
  {
    const bool gen = hp::cols_use_gen(P->real_kind(), n0);
    const int Tb = gen ? hp::gen_symbol_line_threads(P->real_kind(), n0)
                       : hp::symbol_pass_line_threads(P->real_kind(), n0);
    const int Eb = gen ? hp::gen_symbol_elems(P->real_kind()) : n0 / Tb;
    if (Tb > 0 && Eb <= 16) {
      if (gen) P->smask_thr = Tb;
      smask.assign((size_t)P->K * Tb, 0);
      for (int k = 0; k < P->K; ++k)
        for (int j = 0; j < Tb; ++j)
          for (int e2 = 0; e2 < Eb; ++e2) {
            const size_t p = (size_t)j + (size_t)Tb * e2;
            if (p < (size_t)n0 && need[(size_t)k * n0 + p]) smask[(size_t)k * Tb + j] |= (uint16_t)(1u << e2);
          }
    }
  }

  if ((e = upload(P->nodes, nc)) != hipSuccess) return failc(from_hip(e));
  if ((e = upload(P->grpmask, gm)) != hipSuccess) return failc(from_hip(e));
  if ((e = upload(P->slabneed, need)) != hipSuccess) return failc(from_hip(e));
  if ((e = upload(P->storemask, smask)) != hipSuccess) return failc(from_hip(e));
  if ((e = upload(P->lam_ax, lam0)) != hipSuccess) return failc(from_hip(e));
  if ((e = upload(P->lam_in, lamin)) != hipSuccess) return failc(from_hip(e));
  for (int d = 0; d < P->dim; ++d) {
    const int n = P->n[d];
    std::vector<cpx<double>> w(n);
    std::vector<cpx<float>> wf(n);
    for (int m = 0; m < n; ++m) {
      const double ang = 2.0 * M_PI * (double)m / (double)n;
      w[m] = {std::cos(ang), -std::sin(ang)};
      wf[m] = {(float)w[m].re, (float)w[m].im};
    }
    if (P->prec == HP_FP64) {
      if ((e = upload(P->tw64[d], w)) != hipSuccess) return failc(from_hip(e));
    } else {
      if ((e = upload(P->tw32[d], wf)) != hipSuccess) return failc(from_hip(e));
    }
  }
  const size_t fb = (size_t)P->max_nrhs * np * P->fsize();
  if ((e = P->t.alloc(fb)) != hipSuccess) return failc(from_hip(e));
  if ((e = P->fields.alloc(fb * P->K)) != hipSuccess) return failc(from_hip(e));
  // node-field rows that no point uses are never written; keep them finite
  if ((e = hp::launch_fill_zero(P->fields.p, P->fields.bytes, hs)) != hipSuccess) return failc(from_hip(e));
  if ((e = hipStreamSynchronize(hs)) != hipSuccess) return failc(from_hip(e));
  cleanup();
  load_tune(*P);
  *out = P;
  return HP_OK;
}

hp_status hp_plan_query(hp_plan p, hp_plan_info* info) {
  if (!p || !info) return HP_E_INVALID;
  std::memset(info, 0, sizeof(*info));
  info->dim = p->dim;
  for (int d = 0; d < 3; ++d) info->n[d] = p->n[d];
  info->K = p->K;
  info->M = p->M;
  info->Mt = p->Mt;
  info->mo = p->mo;
  info->cmin = p->cmin;
  info->cmax = p->cmax;
  info->zeta_max = p->zmax;
  for (int i = 0; i < 64; ++i) {
    info->cnode[i] = p->cnode[i];
    info->ahat[i] = p->ahat[i];
    info->gamma_re[i] = p->gre[i];
    info->gamma_im[i] = p->gim[i];
  }
  for (int i = 0; i < 65; ++i) info->znode[i] = p->znode[i];
  info->workspace_bytes = p->t.bytes + p->fields.bytes + p->pos.bytes + p->coef64.bytes + p->coef32.bytes;
  info->precision = p->prec;
  info->interp_order = p->order;
  info->m_damp = p->tensor ? 0 : p->Ma;
  info->layer_tensor = p->tensor;
  for (int sl = 0; sl < 5; ++sl) {
    info->tune[sl][0] = p->tune[sl].nthr;
    info->tune[sl][1] = p->tune[sl].tc;
    info->tune[sl][2] = p->tune[sl].order;
    info->tune[sl][3] = p->tune[sl].ng;
  }
  for (int i = 0; i < 64; ++i) info->anode[i] = p->anode[i];
  info->workspace_bytes += p->posa.bytes;
  return HP_OK;
}

}  // extern "C"

namespace {

// u (+)= Q_M v for nrhs <= max_nrhs right-hand sides.
// in_kind/out_kind: 0 = complex128, 1 = complex64.
// ev (optional): 6 events recorded before pass A and after each of the five
// pass slots (A, A', B, M, C; the 3-D-only slots are recorded even when empty).
// reps (profiling only, with acc false): the out-of-place passes A, B and C are
// launched reps times back to back between their events; they read and write
// disjoint buffers, so a repeat recomputes the same result.  The in-place
// middle-axis passes of 3-D grids are launched once.
// Flags of the solver's step and cycle events.  They only tell the host how far
// the device has got; what it then reads (the stop/done flags) is in coherent
// pinned memory that the kernels store to directly, so the events need no
// system-scope fence (an L2 write-back at every step): 11.66 -> 11.58 ms per
// 1024^2 FP64 solve.
#ifndef HP_SOLVER_EVENT_FLAGS
#define HP_SOLVER_EVENT_FLAGS (hipEventDisableTiming | hipEventDisableSystemFence)
#endif
constexpr unsigned kSolverEventFlags = HP_SOLVER_EVENT_FLAGS;

// Right-preconditioned Arnoldi steps on grids of at most kFuseStencilMaxPts
// points compute w = P_N z inside the dot-product sweep (HP_FUSE_STENCIL=0: always
// a separate stencil pass).  Measured per FP64 solve: 256^2 5.06 -> 4.89 ms,
// 512^2 4.20 -> 4.06 ms, 1024^2 11.61 -> 11.55 ms, but 2048^2 65.4 -> 66.5 ms
// (there the sweep's staging of the neighbour rows costs more than the pass).
#ifndef HP_FUSE_STENCIL
#define HP_FUSE_STENCIL 1
#endif
constexpr bool kFuseStencil = HP_FUSE_STENCIL != 0;
constexpr size_t kFuseStencilMaxPts = (size_t)1 << 20;
// Grids of grouped steps (hp_solver_advance_group): up to 1024^2 and 128^3; their
// steps always compute the stencil inside the sweep.
constexpr size_t kGroupMaxPts = (size_t)1 << 21;
#ifndef HP_SOLO_GROUPED
#define HP_SOLO_GROUPED 1
#endif
constexpr bool kSoloGrouped = HP_SOLO_GROUPED != 0;
// FP64 2-D grids with rows of 512, 1024 or 2048 points: the update of Arnoldi step j
// also transforms u_{j+1} along the rows (pass A of step j + 1), whose apply then
// starts at pass B (HP_FUSE_PASS_A=0: separate passes).
#ifndef HP_FUSE_PASS_A
#define HP_FUSE_PASS_A 1
#endif
constexpr bool kFusePassA = HP_FUSE_PASS_A != 0;

// Pass timer: launches recorded per read at most (later ones are not timed).
constexpr size_t kMaxTimedLaunches = 1 << 16;

// Timing events for the next launch of the timed pass on st (nullptr when the
// launch is not timed: a graph capture, or the record is full).
hipError_t timer_events(hp_plan_s* P, hipStream_t st, const hipEvent_t** tev) {
  *tev = nullptr;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return e;
  if (cs != hipStreamCaptureStatusNone || P->timer_n >= kMaxTimedLaunches) return hipSuccess;
  while (P->timer_ev.size() < 2 * (P->timer_n + 1)) {
    hipEvent_t ev;
    if ((e = hipEventCreate(&ev)) != hipSuccess) return e;
    P->timer_ev.push_back(ev);
  }
  *tev = &P->timer_ev[2 * P->timer_n];
  ++P->timer_n;
  return hipSuccess;
}

// Where an apply keeps its intermediate spectrum t and its K node fields: the
// plan's workspace, or (hp_apply_precond_static) the static device array.
struct ApplyWs {
  void* t;
  void* fields;
};

// from_b: pass A's output is already in the plan's t (the fused update of the
// previous Arnoldi step wrote it); the apply starts at pass B.
hipError_t run_apply(hp_plan_s* P, const void* v, int in_kind, size_t in_rs, void* u, int out_kind,
                     size_t out_rs, bool acc, int nrhs, const int* skip, hipStream_t st,
                     hipEvent_t* ev = nullptr, int reps = 1, const ApplyWs* ws = nullptr, bool from_b = false) {
  const int rk = P->real_kind();
  void* const wt = ws ? ws->t : P->t.p;
  if (!ws && !from_b) P->t_owner = nullptr;
  void* const wf = ws ? ws->fields : P->fields.p;
  const size_t np = P->npts;
  hipError_t e;
  const int nl = P->n[P->dim - 1];
  const int rows = (int)(np / nl);
  // the middle-axis slots (2 and 4) only exist in 3-D
  auto mark = [&](int i) {
    return (ev && (P->dim == 3 || (i != 2 && i != 4))) ? hipEventRecord(ev[i], st) : hipSuccess;
  };
  // launch of pass `slot`, with the timer's events when that pass is timed
  auto timed = [&](int slot, auto&& launch) -> hipError_t {
    const hipEvent_t* tev = nullptr;
    if (P->timer_slot == slot && ws == nullptr) {   // the static-workspace path creates no events
      hipError_t e2 = timer_events(P, st, &tev);
      if (e2 != hipSuccess) return e2;
    }
    return launch(tev);
  };
  if ((e = mark(0)) != hipSuccess) return e;
  for (int r = 0; r < (from_b ? 0 : reps); ++r) {
    e = timed(0, [&](const hipEvent_t* tev) {
      return hp::launch_rows_fwd(rk, in_kind, nl, v, wt, rows, in_rs, np, nrhs, P->tw(P->dim - 1), skip,
                                 P->tune[0], st, tev);
    });
    if (e != hipSuccess) return e;
  }
  if ((e = mark(1)) != hipSuccess) return e;
  if (P->dim == 3) {   // forward along the middle axis, in place
    hp::ColsArgs m{};
    m.real_kind = rk; m.n = P->n[1]; m.dir = -1; m.mode = 0;
    m.in = wt; m.out = wt; m.S = P->n[2]; m.outer = P->n[0]; m.nfields = 1; m.nrhs = nrhs;
    m.in_rs = np; m.out_rs = np; m.in_fs = np; m.out_fs = np; m.tw = P->tw(1); m.skip = skip;
    m.tune = P->tune[1];
    if ((e = timed(1, [&](const hipEvent_t* tev) { m.tev = tev; return hp::launch_cols(m, st); })) != hipSuccess)
      return e;
  }
  if ((e = mark(2)) != hipSuccess) return e;
  hp::ColsArgs b{};
  b.real_kind = rk; b.n = P->n[0]; b.dir = -1; b.mode = 1;
  b.in = wt; b.out = wf; b.S = (int)(np / P->n[0]); b.outer = 1; b.nfields = 1; b.nrhs = nrhs;
  b.in_rs = np; b.out_rs = np * P->K; b.in_fs = np; b.out_fs = np; b.tw = P->tw(0); b.skip = skip;
  b.lam_ax = (const double*)P->lam_ax.p; b.lam_in = (const double*)P->lam_in.p;
  b.nodes = (const hp::NodeConst*)P->nodes.p; b.K = P->K; b.scale = 1.0 / (double)np;
  b.store_mask = (const uint16_t*)P->storemask.p;
  b.store_mask_thr = P->smask_thr;
  b.store_need = (const uint8_t*)P->slabneed.p;
  b.tune = P->tune[2];
  for (int r = 0; r < reps; ++r)
    if ((e = timed(2, [&](const hipEvent_t* tev) { b.tev = tev; return hp::launch_cols(b, st); })) != hipSuccess)
      return e;
  if ((e = mark(3)) != hipSuccess) return e;
  if (P->dim == 3) {   // inverse along the middle axis for the K fields, in place
    hp::ColsArgs m{};
    m.real_kind = rk; m.n = P->n[1]; m.dir = +1; m.mode = 0;
    m.in = wf; m.out = wf; m.S = P->n[2]; m.outer = P->n[0]; m.nfields = P->K; m.nrhs = nrhs;
    m.in_rs = np * P->K; m.out_rs = np * P->K; m.in_fs = np; m.out_fs = np; m.tw = P->tw(1); m.skip = skip;
    m.slab_need = (const uint8_t*)P->slabneed.p;
    m.tune = P->tune[3];
    if ((e = timed(3, [&](const hipEvent_t* tev) { m.tev = tev; return hp::launch_cols(m, st); })) != hipSuccess)
      return e;
  }
  if ((e = mark(4)) != hipSuccess) return e;
  hp::CombineArgs c{};
  c.real_kind = rk; c.out_kind = out_kind; c.accumulate = acc ? 1 : 0; c.n = nl;
  c.fields = wf; c.fs = np; c.frs = np * P->K; c.pos = (const double*)P->pos.p;
  c.grpmask = (const uint64_t*)P->grpmask.p; c.rowmask = (const uint64_t*)P->rowmask.p; c.out = u; c.out_rs = out_rs; c.rows = rows; c.K = P->K;
  c.M = P->M; c.Mt = P->Mt; c.mo = P->mo; c.nrhs = nrhs; c.tw = P->tw(P->dim - 1); c.skip = skip;
  c.order = P->order; c.lag = (const double*)P->lagtab.p;
  c.posa = (const double*)P->posa.p; c.Ma = P->Ma;
  c.tune = P->tune[4];
  for (int r = 0; r < (acc ? 1 : reps); ++r)
    if ((e = timed(4, [&](const hipEvent_t* tev) { c.tev = tev; return hp::launch_combine(c, st); })) != hipSuccess)
      return e;
  return mark(5);
}

// Per-launch time (ms) of each pass slot (A, A', B, M, C; 0 for slots a 2-D grid does
// not have): one plain apply first (fills the intermediate buffers and warms the
// caches), then every out-of-place pass reps times back to back between a pair of
// events, so that an event pair brackets a run of launches of one kernel and the
// per-launch figure is that kernel's duration (the in-place 3-D middle-axis passes run
// once).
hipError_t time_passes(hp_plan_s* p, const void* v, void* u, int nrhs, int reps, double* ms, hipStream_t st) {
  const int kind = p->prec == HP_FP64 ? 0 : 1;
  hipEvent_t ev[6];
  for (int i = 0; i < 6; ++i) {
    hipError_t e = hipEventCreate(&ev[i]);
    if (e != hipSuccess) {
      for (int k = 0; k < i; ++k) (void)hipEventDestroy(ev[k]);
      return e;
    }
  }
  double acc[5] = {0, 0, 0, 0, 0};
  hipError_t err = run_apply(p, v, kind, p->npts, u, kind, p->npts, false, nrhs, nullptr, st);
  if (err == hipSuccess) err = run_apply(p, v, kind, p->npts, u, kind, p->npts, false, nrhs, nullptr, st, ev, reps);
  if (err == hipSuccess) err = hipEventSynchronize(ev[5]);
  const int slots3[5][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 4}, {4, 5}};
  const int slots2[5][2] = {{0, 1}, {-1, -1}, {1, 3}, {-1, -1}, {3, 5}};
  const int count[5] = {reps, 1, reps, 1, reps};
  for (int i = 0; i < 5 && err == hipSuccess; ++i) {
    const int a = p->dim == 3 ? slots3[i][0] : slots2[i][0], b = p->dim == 3 ? slots3[i][1] : slots2[i][1];
    if (a < 0) continue;
    float t = 0;
    err = hipEventElapsedTime(&t, ev[a], ev[b]);
    acc[i] = (double)t / count[i];
  }
  for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
  for (int i = 0; i < 5; ++i) ms[i] = acc[i];
  return err;
}

// Tuning cache: the file named by HP_TUNE_CACHE, one line per pass choice,
//   hp-tune <dim> <n0> <n1> <n2> <precision> <K> <slot> <nthr> <tc> <order> <ng>
// appended by hp_plan_autotune and read (later lines win) when a plan is created.
void load_tune(hp_plan_s& P) {
  const char* path = std::getenv("HP_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char tag[16];
  int d, n0, n1, n2, prec, K, slot, nthr, tc, order, ng;
  while (std::fscanf(f, "%15s %d %d %d %d %d %d %d %d %d %d %d", tag, &d, &n0, &n1, &n2, &prec, &K, &slot, &nthr, &tc,
                     &order, &ng) == 12) {
    if (std::strcmp(tag, "hp-tune") != 0 || d != P.dim || n0 != P.n[0] || n1 != P.n[1] || n2 != P.n[2] ||
        prec != P.prec || K != P.K || slot < 0 || slot > 4)
      continue;
    P.tune[slot] = hp::PassTune{std::max(0, nthr), std::max(0, tc), std::max(0, order), std::max(0, ng)};
  }
  std::fclose(f);
}

void save_tune(const hp_plan_s& P) {
  const char* path = std::getenv("HP_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  for (int sl = 0; sl < 5; ++sl) {
    const hp::PassTune& t = P.tune[sl];
    std::fprintf(f, "hp-tune %d %d %d %d %d %d %d %d %d %d %d\n", P.dim, P.n[0], P.n[1], P.n[2], P.prec, P.K, sl, t.nthr,
                 t.tc, t.order, t.ng);
  }
  std::fclose(f);
}

// Algorithmic bytes of each pass for one launch over nrhs fields.
void pass_bytes(const hp_plan_s* P, int nrhs, int in_bytes, int out_bytes, double* b) {
  const double np = (double)P->npts, sf = (double)P->fsize(), nr = nrhs;
  const double S = np / P->n[0];
  b[0] = nr * np * (in_bytes + sf);
  b[1] = P->dim == 3 ? nr * np * 2 * sf : 0.0;
  b[2] = nr * (np * sf + P->slabs_used * S * sf);
  b[3] = P->dim == 3 ? nr * P->slabs_used * S * 2 * sf : 0.0;
  b[4] = nr * (np * (8.0 + out_bytes) + P->rows_used * P->n[P->dim - 1] * sf);
}

hp::StencilArgs stencil_args(hp_plan_s* P, int kind, const void* u, size_t u_rs, void* y, size_t y_rs,
                             const void* f, int nrhs, const int* skip) {
  hp::StencilArgs s{};
  s.kind = kind;
  s.dim = P->dim;
  for (int d = 0; d < 3; ++d) {
    s.n[d] = P->n[d];
    const double h = P->len[d] / P->n[d];
    s.ih2[d] = d < P->dim ? 1.0 / (h * h) : 0.0;
  }
  s.u = u; s.u_rs = u_rs; s.y = y; s.y_rs = y_rs; s.f = f;
  s.coef = (kind == 1 || kind == 2) ? P->coef32.p : P->coef64.p;
  s.nrhs = nrhs;
  s.skip = skip;
  return s;
}

hipError_t run_stencil(hp_plan_s* P, int kind, const void* u, size_t u_rs, void* y, size_t y_rs,
                       const void* f, int nrhs, const int* skip, hipStream_t st) {
  return hp::launch_stencil(stencil_args(P, kind, u, u_rs, y, y_rs, f, nrhs, skip), st);
}

}  // namespace

extern "C" {

hp_status hp_apply_precond(hp_plan p, const void* v, void* u, int nrhs, void* stream) {
  if (!p || !v || !u || nrhs < 0) return HP_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  const size_t fs = p->fsize();
  const int kind = p->prec == HP_FP64 ? 0 : 1;
  for (int r0 = 0; r0 < nrhs; r0 += p->max_nrhs) {
    const int nr = std::min(p->max_nrhs, nrhs - r0);
    const char* vi = (const char*)v + (size_t)r0 * p->npts * fs;
    char* uo = (char*)u + (size_t)r0 * p->npts * fs;
    HP_TRY(run_apply(p, vi, kind, p->npts, uo, kind, p->npts, false, nr, nullptr, st));
  }
  return HP_OK;
}

hp_status hp_apply_precond_static(hp_plan p, const void* v, void* u, int nrhs, void* stream) {
  if (!p || !v || !u || nrhs < 0) return HP_E_INVALID;
  const size_t fb = p->npts * p->fsize();                 // one field
  auto round256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
  auto need = [&](size_t nr) { return round256(nr * fb) + nr * fb * (size_t)p->K; };
  if (need(1) > HP_STATIC_SCRATCH_BYTES) {
    std::snprintf(g_last_error, sizeof(g_last_error),
                  "hp_apply_precond_static: one field needs %zu bytes ((1 + K) N^d S with K = %d), the static "
                  "workspace holds %zu",
                  need(1), p->K, (size_t)HP_STATIC_SCRATCH_BYTES);
    return HP_E_INVALID;
  }
  if (nrhs == 0) return HP_OK;
  void* base = nullptr;
  HP_TRY(hp::static_scratch(&base));
  size_t chunk = 1;
  while (chunk < (size_t)nrhs && need(chunk + 1) <= HP_STATIC_SCRATCH_BYTES) ++chunk;
  const ApplyWs ws{base, (char*)base + round256(chunk * fb)};
  hipStream_t st = (hipStream_t)stream;
  const int kind = p->prec == HP_FP64 ? 0 : 1;
  for (size_t r0 = 0; r0 < (size_t)nrhs; r0 += chunk) {
    const int nr = (int)std::min(chunk, (size_t)nrhs - r0);
    const char* vi = (const char*)v + r0 * fb;
    char* uo = (char*)u + r0 * fb;
    HP_TRY(run_apply(p, vi, kind, p->npts, uo, kind, p->npts, false, nr, nullptr, st, nullptr, 1, &ws));
  }
  return HP_OK;
}

hp_status hp_matvec(hp_plan p, const void* u, void* y, int nrhs, void* stream) {
  if (!p || !u || !y || nrhs < 0) return HP_E_INVALID;
  if (u == y) return HP_E_INVALID;
  if (nrhs == 0) return HP_OK;
  const int kind = p->prec == HP_FP64 ? 0 : 1;
  HP_TRY(run_stencil(p, kind, u, p->npts, y, p->npts, nullptr, nrhs, nullptr, (hipStream_t)stream));
  return HP_OK;
}

}  // extern "C"

// Krylov workspace of one batch of right-hand sides: the FP64 basis, the
// preconditioned vector, the solution update, the per-right-hand-side state,
// partial sums, device flags and their pinned host copies.
struct SolverWs {
  static constexpr int kLag = 3;   // Arnoldi steps a session keeps in flight
  DevBuf V, z, tvec, state, part, flags;
  int* pinned = nullptr;           // [0, n): done (host copy), [n, 2n): cycle ended (host copy)
  hipEvent_t step_ev[kLag + 1] = {};
  hipEvent_t cyc_ev = nullptr;
  int restart = 0, nrhs = 0;
  // Arnoldi steps captured as HIP graphs (small grids), one per step index j, for the
  // session configuration `graph_key` (plan, side, right-hand sides, restart, tuning
  // generation); captured on a private stream, launched on the session's stream
  hipGraphExec_t step_graph[hp::kMaxRestart] = {};
  hipStream_t cap_st = nullptr;
  uint64_t graph_key = 0;
  void drop_graphs() {
    for (hipGraphExec_t& g : step_graph) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
    graph_key = 0;
  }

  static size_t bytes(size_t np, size_t fsize, int restart, int nrhs) {
    const size_t n = (size_t)nrhs;
    return n * ((size_t)(restart + 1) * np * 16 + np * fsize + np * 16 + sizeof(hp::KState) +
                (size_t)hp::kRedBlocks * hp::kPartSlots * 16 + 3 * sizeof(int));
  }
  hipError_t ensure(size_t np, size_t fsize, int r, int n) {
    if (restart >= r && nrhs >= n) return hipSuccess;
    r = std::max(r, restart);
    n = std::max(n, nrhs);
    drop_graphs();   // the captured steps point into the buffers about to be replaced
    hipError_t e;
    if ((e = V.alloc((size_t)n * (r + 1) * np * 16)) != hipSuccess) return e;
    if ((e = z.alloc((size_t)n * np * fsize)) != hipSuccess) return e;
    if ((e = tvec.alloc((size_t)n * np * 16)) != hipSuccess) return e;
    if ((e = state.alloc((size_t)n * sizeof(hp::KState))) != hipSuccess) return e;
    if ((e = part.alloc((size_t)n * hp::kRedBlocks * hp::kPartSlots * 16)) != hipSuccess) return e;
    if ((e = flags.alloc((size_t)n * 3 * sizeof(int))) != hipSuccess) return e;
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    if ((e = hipHostMalloc((void**)&pinned, (size_t)n * 2 * sizeof(int), hipHostMallocCoherent)) != hipSuccess)
      return e;
    std::memset(pinned, 0, (size_t)n * 2 * sizeof(int));
    for (hipEvent_t& ev : step_ev)
      if (!ev && (e = hipEventCreateWithFlags(&ev, kSolverEventFlags)) != hipSuccess) return e;
    if (!cyc_ev && (e = hipEventCreateWithFlags(&cyc_ev, kSolverEventFlags)) != hipSuccess) return e;
    restart = r;
    nrhs = n;
    return hipSuccess;
  }
  void release() {
    drop_graphs();
    if (cap_st) (void)hipStreamDestroy(cap_st);
    cap_st = nullptr;
    for (DevBuf* b : {&V, &z, &tvec, &state, &part, &flags}) b->release();
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    for (hipEvent_t& ev : step_ev) {
      if (ev) (void)hipEventDestroy(ev);
      ev = nullptr;
    }
    if (cyc_ev) (void)hipEventDestroy(cyc_ev);
    cyc_ev = nullptr;
    restart = nrhs = 0;
  }
};

// Inverse operators of hp_arnoldi (HP_LEFT_INVERSE, HP_NONE_INVERSE) and the
// restarted GMRES of their inner solves.
constexpr int kLeftInverse = 3, kNoneInverse = 4;
constexpr int kInnerRestart = 64, kInnerCycles = 50;
constexpr double kInnerRtol = 1e-10;

// A resumable restarted-GMRES solve of nrhs right-hand sides on one stream.
// The Krylov state stays on the device; the host only enqueues work and reads
// two pinned flag arrays the kernels publish (converged, cycle ended), so that
// several sessions can progress concurrently on separate streams.
struct Session {
  hp_plan_s* P = nullptr;
  SolverWs* W = nullptr;
  const cpx<double>* f = nullptr;
  cpx<double>* x = nullptr;
  int nrhs = 0;
  hp_solve_opts o{};
  hipStream_t st = nullptr;
  hp::KrylovArgs K{};
  size_t vrs = 0;
  enum Phase { kIdle, kCycleStart, kArnoldi, kFinished } phase = kIdle;
  int cycles_run = 0, j = 0;
  bool throttle = true;
  // one Arnoldi process from f itself (every side): no preconditioner on the start,
  // no cycle end, the basis stays in the workspace
  bool arnoldi_only = false;
  // left side: f is the preconditioned right-hand side itself (the system Q P x = f)
  bool rhs_prec = false;
  bool inner_failed = false;   // an inner solve of an inverse operator stopped above its tolerance
  // Arnoldi steps as HIP graphs: for grids where a step is too short to hide the
  // launches (the same threshold as `throttle`), when HP_STEP_GRAPHS=1
  bool use_graphs = false;
  hp_status status = HP_OK;

  hipError_t start(const cpx<double>* f_, cpx<double>* x_, hipStream_t s) {
    f = f_;
    x = x_;
    st = s;
    const size_t np = P->npts;
    vrs = (size_t)(W->restart + 1) * np;
    K = hp::KrylovArgs{};
    K.V = (cpx<double>*)W->V.p;
    K.npts = np;
    K.vrs = vrs;
    K.state = (hp::KState*)W->state.p;
    K.part = (cpx<double>*)W->part.p;
    K.skip_step = (int*)W->flags.p;
    K.done = (int*)W->flags.p + W->nrhs;
    K.host_done = W->pinned;
    K.host_stop = W->pinned + W->nrhs;
    K.nrhs = nrhs;
    K.restart = o.restart;
    cycles_run = 0;
    j = 0;
    hipError_t e;
    if ((e = hp::launch_fill_zero(W->flags.p, W->flags.bytes, st)) != hipSuccess) return e;
    if (o.side == HP_LEFT && !arnoldi_only && !rhs_prec) {   // the stopping test uses ||Q f||; ||f|| for the reported true residual
      cpx<double>* qf = (cpx<double>*)W->tvec.p;
      if ((e = run_apply(P, f, 0, np, qf, 0, np, false, nrhs, nullptr, st)) != hipSuccess) return e;
      if ((e = hp::launch_fnorm(K, qf, np, o.rtol, st)) != hipSuccess) return e;
      if ((e = hp::launch_plain_norm(K, f, np, 0, st)) != hipSuccess) return e;
    } else if ((e = hp::launch_fnorm(K, f, np, o.rtol, st)) != hipSuccess) {
      return e;
    }
    return enqueue_cycle_start();
  }

  // residual r = f - P_N x into v_0 (Q r for a left-preconditioned solve), its
  // norm and the convergence test
  hipError_t enqueue_cycle_start() {
    hipError_t e;
    if (o.side == HP_LEFT && rhs_prec) {   // r = f - Q P x
      const size_t np = P->npts;
      cpx<double>* px = (cpx<double>*)W->tvec.p;
      if ((e = run_stencil(P, 0, x, np, px, np, nullptr, nrhs, K.done, st)) != hipSuccess) return e;
      if ((e = run_apply(P, px, 0, np, K.V, 0, vrs, false, nrhs, K.done, st)) != hipSuccess) return e;
      if ((e = hp::launch_rsub(f, np, K.V, vrs, np, nrhs, K.done, st)) != hipSuccess) return e;
      if ((e = hp::launch_cycle_start(K, o.rtol, st)) != hipSuccess) return e;
      if ((e = hipEventRecord(W->cyc_ev, st)) != hipSuccess) return e;
      phase = kCycleStart;
      return hipSuccess;
    }
    if ((e = run_stencil(P, 3, x, P->npts, K.V, vrs, f, nrhs, K.done, st)) != hipSuccess) return e;
    if (o.side == HP_LEFT && !arnoldi_only &&
        (e = run_apply(P, K.V, 0, vrs, K.V, 0, vrs, false, nrhs, K.done, st)) != hipSuccess)
      return e;
    if ((e = hp::launch_cycle_start(K, o.rtol, st)) != hipSuccess) return e;
    if ((e = hipEventRecord(W->cyc_ev, st)) != hipSuccess) return e;
    phase = kCycleStart;
    return hipSuccess;
  }

  // The kernels of Arnoldi step j on stream s (a fixed sequence for given j).
  hipError_t step_kernels(hipStream_t s) {
    const size_t np = P->npts;
    const int mixed = P->prec == HP_MIXED;
    cpx<double>* vj = K.V + (size_t)j * np;
    cpx<double>* vj1 = K.V + (size_t)(j + 1) * np;
    hipError_t e;
    if (o.side == HP_NONE) {          // w = P_N u_j (plain GMRES, FP64)
      if ((e = run_stencil(P, 0, vj, vrs, vj1, vrs, nullptr, nrhs, K.skip_step, s)) != hipSuccess) return e;
    } else if (o.side == HP_LEFT) {   // w = Q P_N u_j (P_N in FP64)
      cpx<double>* pv = (cpx<double>*)W->tvec.p;
      if ((e = run_stencil(P, 0, vj, vrs, pv, np, nullptr, nrhs, K.skip_step, s)) != hipSuccess) return e;
      if ((e = run_apply(P, pv, 0, np, vj1, 0, vrs, false, nrhs, K.skip_step, s)) != hipSuccess) return e;
    } else {                          // w = P_N Q u_j, the stencil fused with the sweep
      // a step the grouped kernels take runs them (as a group of one), so that it gives
      // bitwise the result of the same step inside a grouped launch
      hp::GroupMember gm;
      if (kSoloGrouped && group_member(&gm)) return hp::launch_group_step(&gm, 1, s);
      // step 0 of a cycle transforms u_0 itself; a later step finds it in t when its
      // own previous update was the last thing enqueued to write t
      const bool from_b = fused_pass_a() && j > 0 && P->t_owner == this && P->t_step == j;
      if ((e = run_apply(P, vj, 0, vrs, W->z.p, mixed ? 1 : 0, np, false, nrhs, K.skip_step, s, nullptr, 1, nullptr,
                         from_b)) != hipSuccess)
        return e;
      if (kFuseStencil && np <= kFuseStencilMaxPts) {
        const hp::StencilArgs sa = stencil_args(P, mixed ? 2 : 0, W->z.p, np, vj1, vrs, nullptr, nrhs, K.skip_step);
        if ((e = hp::launch_arnoldi_dots_stencil(K, j, sa, s)) != hipSuccess) return e;
        return update(s);
      }
      if ((e = run_stencil(P, mixed ? 2 : 0, W->z.p, np, vj1, vrs, nullptr, nrhs, K.skip_step, s)) != hipSuccess)
        return e;
    }
    if ((e = hp::launch_arnoldi_dots(K, j, s)) != hipSuccess) return e;
    return update(s);
  }

  // The right-preconditioned steps of FP64 2-D grids whose rows the fused update
  // transforms (not in captured step graphs: a replay cannot see who wrote t last).
  bool fused_pass_a() const {
    return kFusePassA && !use_graphs && o.side == HP_RIGHT &&
           hp::update_rows_fits(P->real_kind(), P->dim, P->n[P->dim - 1]);
  }
  hipError_t update(hipStream_t s) {
    if (!fused_pass_a()) return hp::launch_arnoldi_update(K, j, s);
    hipError_t e = hp::launch_arnoldi_update_rows(K, j, P->t.p, P->n[P->dim - 1], P->tw(P->dim - 1), s);
    P->t_owner = e == hipSuccess ? this : nullptr;
    P->t_step = j + 1;
    return e;
  }

  // Step j as a graph: captured once per workspace configuration on the private
  // stream (nothing runs during capture), then launched on the session's stream.
  hipError_t launch_step_graph() {
    hipError_t e;
    const uint64_t key = graph_key_of();
    if (W->graph_key != key) {
      W->drop_graphs();
      W->graph_key = key;
    }
    hipGraphExec_t& ge = W->step_graph[j];
    if (!ge) {
      if (!W->cap_st && (e = hipStreamCreateWithFlags(&W->cap_st, hipStreamNonBlocking)) != hipSuccess) return e;
      if ((e = hipStreamBeginCapture(W->cap_st, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
      hipError_t ek = step_kernels(W->cap_st);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(W->cap_st, &g);
      if (ek != hipSuccess) e = ek;
      if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        ge = nullptr;
        return e;
      }
    }
    return hipGraphLaunch(ge, st);
  }

  uint64_t graph_key_of() const {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
    mix((uint64_t)(uintptr_t)P);
    mix((uint64_t)o.side);
    mix((uint64_t)nrhs);
    mix((uint64_t)W->restart);
    mix((uint64_t)o.restart);
    mix((uint64_t)P->tune_gen);
    return h == 0 ? 1 : h;
  }

  hipError_t enqueue_step() {
    hipError_t e;
    if (o.side == kLeftInverse || o.side == kNoneInverse) {   // w = (Q P_N)^{-1} u_j or P_N^{-1} u_j
      const size_t np = P->npts;
      if ((e = inner_solve(K.V + (size_t)j * np, K.V + (size_t)(j + 1) * np)) != hipSuccess) return e;
      if ((e = hp::launch_arnoldi_dots(K, j, st)) != hipSuccess) return e;
      if ((e = hp::launch_arnoldi_update(K, j, st)) != hipSuccess) return e;
    } else if (use_graphs) {
      if ((e = launch_step_graph()) != hipSuccess) return e;
    } else if ((e = step_kernels(st)) != hipSuccess) {
      return e;
    }
    if ((e = hipEventRecord(W->step_ev[j % (SolverWs::kLag + 1)], st)) != hipSuccess) return e;
    ++j;
    return hipSuccess;
  }

  // out = A^{-1} in for the inverse operators of hp_arnoldi, by a blocking restarted
  // GMRES on the same stream with the plan's inner workspace: Q P_N x = in (left
  // side, right-hand side taken as given), or P_N x = in preconditioned on the right
  hipError_t inner_solve(const cpx<double>* in, cpx<double>* out) {
    hipError_t e;
    if ((e = hp::launch_fill_zero(out, P->npts * sizeof(cpx<double>), st)) != hipSuccess) return e;
    // the outer process has stopped (an invariant subspace): its remaining steps are void
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (all(K.host_stop)) return hipSuccess;
    Session I;
    I.P = P;
    I.W = P->inner_ws_ptr;
    I.nrhs = 1;
    I.o = hp_solve_opts{kInnerRestart, kInnerCycles, kInnerRtol, o.side == kLeftInverse ? HP_LEFT : HP_RIGHT};
    I.rhs_prec = o.side == kLeftInverse;
    I.throttle = throttle;
    if ((e = I.start(in, out, st)) != hipSuccess) return e;
    if ((e = I.advance(1 << 30, true)) != hipSuccess) return e;
    if (!I.all(I.K.host_done)) inner_failed = true;
    return hipSuccess;
  }

  // x += Q (V_k y), then the next cycle start
  hipError_t enqueue_cycle_end() {
    hipError_t e;
    if ((e = hp::launch_backsolve(K, st)) != hipSuccess) return e;
    if (o.side != HP_RIGHT) {   // x += V_k y
      if ((e = hp::launch_lincomb(K, x, P->npts, true, st)) != hipSuccess) return e;
    } else {
      if ((e = hp::launch_lincomb(K, (cpx<double>*)W->tvec.p, P->npts, false, st)) != hipSuccess) return e;
      if ((e = run_apply(P, W->tvec.p, 0, P->npts, x, 0, P->npts, true, nrhs, K.done, st)) != hipSuccess) return e;
    }
    ++cycles_run;
    return enqueue_cycle_start();
  }

  static bool ready(hipEvent_t ev, bool block, hipError_t& e) {
    if (block) {
      e = hipEventSynchronize(ev);
      return e == hipSuccess;
    }
    e = hipEventQuery(ev);
    if (e == hipErrorNotReady) {
      e = hipSuccess;
      return false;
    }
    return e == hipSuccess;
  }

  bool all(const int* flags) const {
    for (int r = 0; r < nrhs; ++r)
      if (!__atomic_load_n(&flags[r], __ATOMIC_ACQUIRE)) return false;
    return true;
  }

  // Enqueue the cycle transitions that are due, up to the point where the next
  // action is an Arnoldi step (kPollStep), needs a result the device has not
  // produced yet (kPollWait; only with block = false) or the solve has ended
  // (kPollDone).
  enum Poll { kPollStep, kPollWait, kPollDone };
  Poll poll(bool block, hipError_t& e) {
    e = hipSuccess;
    while (phase != kFinished) {
      if (phase == kCycleStart) {
        if (!ready(W->cyc_ev, block, e)) return kPollWait;
        if (all(K.host_done) || cycles_run >= o.max_cycles) {
          phase = kFinished;
          if (o.side == HP_LEFT && !rhs_prec) {   // the true residual of the returned x
            cpx<double>* r = (cpx<double>*)W->tvec.p;
            if ((e = run_stencil(P, 3, x, P->npts, r, P->npts, f, nrhs, nullptr, st)) != hipSuccess) return kPollWait;
            if ((e = hp::launch_plain_norm(K, r, P->npts, 1, st)) != hipSuccess) return kPollWait;
          }
          return kPollDone;
        }
        if ((e = hp::launch_scale_v0(K, st)) != hipSuccess) return kPollWait;
        j = 0;
        phase = kArnoldi;
        continue;
      }
      // kArnoldi
      if (j >= o.restart) {
        if (arnoldi_only) {
          phase = kFinished;
          return kPollDone;
        }
        if ((e = enqueue_cycle_end()) != hipSuccess) return kPollWait;
        continue;
      }
      if (j >= SolverWs::kLag && (throttle || !block)) {
        // keep at most kLag steps in flight; end the cycle once every
        // right-hand side has ended it
        if (!ready(W->step_ev[(j - SolverWs::kLag) % (SolverWs::kLag + 1)], block, e)) return kPollWait;
        if (all(K.host_stop)) {
          if (arnoldi_only) {
            phase = kFinished;
            return kPollDone;
          }
          if ((e = enqueue_cycle_end()) != hipSuccess) return kPollWait;
          continue;
        }
      }
      return kPollStep;
    }
    return kPollDone;
  }

  // Enqueue up to max_steps Arnoldi steps (and the cycle transitions they
  // reach).  block = false never waits: it returns when the next action needs
  // a result the device has not produced yet.
  hipError_t advance(int max_steps, bool block) {
    hipError_t e = hipSuccess;
    int steps = 0;
    while (true) {
      if (poll(block, e) != kPollStep || e != hipSuccess) return e;
      if (steps >= max_steps) return hipSuccess;
      if ((e = enqueue_step()) != hipSuccess) return e;
      ++steps;
    }
  }

  // This session's current Arnoldi step as a member of a grouped launch, when the
  // grouped kernels take it: one right-hand side, right preconditioning, the FP32
  // preconditioner, grids of at most kGroupMaxPts points with power-of-two lines the
  // grouped passes cover, and the combine's built-in workgroup shape.
  bool group_member(hp::GroupMember* g) const {
    if (o.side != HP_RIGHT || arnoldi_only || nrhs != 1 || P->prec != HP_MIXED || P->tune[4].ng > 1 ||
        W->z.p == nullptr || P->npts > kGroupMaxPts)
      return false;
    hp::GroupMember m{};
    m.dim = P->dim;
    for (int d = 0; d < 3; ++d) m.n[d] = P->n[d];
    m.npts = P->npts;
    m.K = P->K;
    m.M = P->M;
    m.Mt = P->Mt;
    m.mo = P->mo;
    m.order = P->order;
    m.Ma = P->Ma;
    m.interp = P->Ma >= 2 ? 2 : (P->order >= 2 ? 1 : 0);
    m.scale = 1.0 / (double)P->npts;
    for (int d = 0; d < P->dim; ++d) m.tw[d] = P->tw(d);
    m.lam_ax = (const double*)P->lam_ax.p;
    m.lam_in = (const double*)P->lam_in.p;
    m.nodes = (const hp::NodeConst*)P->nodes.p;
    m.store_mask = (const uint16_t*)P->storemask.p;
    m.slab_need = (const uint8_t*)P->slabneed.p;
    m.pos = (const double*)P->pos.p;
    m.posa = (const double*)P->posa.p;
    m.grpmask = (const uint64_t*)P->grpmask.p;
    m.rowmask = (const uint64_t*)P->rowmask.p;
    m.lag = (const double*)P->lagtab.p;
    m.coef32 = P->coef32.p;
    for (int d = 0; d < 3; ++d) {
      const double h = P->len[d] / P->n[d];
      m.ih2[d] = d < P->dim ? 1.0 / (h * h) : 0.0;
    }
    m.t = P->t.p;
    m.fields = P->fields.p;
    m.z = W->z.p;
    m.V = K.V;
    m.state = K.state;
    m.part = K.part;
    m.skip_step = K.skip_step;
    m.host_stop = K.host_stop;
    m.j = j;
    m.restart = o.restart;
    m.ng_b = P->tune[2].ng;
    if (!hp::group_member_ok(m)) return false;
    *g = m;
    return true;
  }

  // After a grouped launch that included this session's step j.
  hipError_t stepped_in_group() {
    hipError_t e = hipEventRecord(W->step_ev[j % (SolverWs::kLag + 1)], st);
    if (e != hipSuccess) return e;
    ++j;
    return hipSuccess;
  }

  // After kFinished: per right-hand side results (blocking copy of the states).
  hp_status collect(hp_solve_info* info) {
    std::vector<hp::KState> hs(nrhs);
    HP_TRY(hipMemcpyAsync(hs.data(), W->state.p, (size_t)nrhs * sizeof(hp::KState), hipMemcpyDeviceToHost, st));
    HP_TRY(hipStreamSynchronize(st));
    hp_status ret = HP_OK;
    for (int r = 0; r < nrhs; ++r) {
      const bool ok = W->pinned[r] != 0;
      info[r].iters = hs[r].iters;
      // the device counts a cycle when its start finds the tolerance unmet; the start
      // that follows the last allowed cycle is counted there but never run
      info[r].cycles = std::min(hs[r].cycles, o.max_cycles);
      info[r].rel_true_residual = o.side == HP_LEFT && !rhs_prec ? hs[r].relres_plain : hs[r].relres;
      info[r].rel_prec_residual = hs[r].relres;
      if (!std::isfinite(hs[r].relres)) {   // a non-finite right-hand side or residual
        info[r].status = HP_E_NONFINITE;
        ret = HP_E_NONFINITE;
        continue;
      }
      info[r].status = ok ? HP_OK : HP_E_NOT_CONVERGED;
      if (!ok && ret == HP_OK) ret = HP_E_NOT_CONVERGED;
    }
    return ret;
  }
};

struct hp_solver_s {
  Session sess;
  SolverWs ws;
};

void hp_plan_s::release_solver_ws() {
  for (SolverWs** w : {&solver_ws_ptr, &inner_ws_ptr}) {
    if (*w) {
      (*w)->release();
      delete *w;
    }
    *w = nullptr;
  }
}

static hp_status solve_batch(hp_plan_s* P, const cpx<double>* f, cpx<double>* x, int nrhs,
                             const hp_solve_opts& o, hp_solve_info* info, hipStream_t st) {
  if (!P->solver_ws_ptr) {
    P->solver_ws_ptr = new (std::nothrow) SolverWs();
    if (!P->solver_ws_ptr) return HP_E_NOMEM;
  }
  HP_TRY(P->solver_ws_ptr->ensure(P->npts, P->fsize(), o.restart, nrhs));
  P->arnoldi_k = -1;
  Session S;
  S.P = P;
  S.W = P->solver_ws_ptr;
  S.nrhs = nrhs;
  S.o = o;
  // small problems: a step is too short to hide a host round trip, enqueue freely,
  // and launch each step as one graph
  S.throttle = P->npts * (size_t)nrhs >= ((size_t)1 << 18);
  S.use_graphs = !S.throttle && step_graphs_enabled();
  HP_TRY(S.start(f, x, st));
  HP_TRY(S.advance(1 << 30, true));
  return S.collect(info);
}

extern "C" {

hp_status hp_arnoldi(hp_plan p, const void* v0, int m, int side, void* H, int* steps, void* stream) {
  if (!p || !v0 || !H || !steps || m < 1 || m > hp::kMaxRestart || side < HP_RIGHT || side > kNoneInverse)
    return HP_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  if (!p->solver_ws_ptr) {
    p->solver_ws_ptr = new (std::nothrow) SolverWs();
    if (!p->solver_ws_ptr) return HP_E_NOMEM;
  }
  HP_TRY(p->solver_ws_ptr->ensure(p->npts, p->fsize(), m, 1));
  if (side >= kLeftInverse) {
    if (!p->inner_ws_ptr) {
      p->inner_ws_ptr = new (std::nothrow) SolverWs();
      if (!p->inner_ws_ptr) return HP_E_NOMEM;
    }
    HP_TRY(p->inner_ws_ptr->ensure(p->npts, p->fsize(), kInnerRestart, 1));
  }
  p->arnoldi_k = -1;
  DevBuf x0;   // the starting guess of the cycle (zero): its residual is v0
  HP_TRY(x0.alloc(p->npts * 16));
  HP_TRY(hp::launch_fill_zero(x0.p, x0.bytes, st));
  // m steps under a tolerance no residual meets: only an invariant subspace ends it early
  const hp_solve_opts o{m, 1, 1e-300, side};
  Session S;
  S.P = p;
  S.W = p->solver_ws_ptr;
  S.nrhs = 1;
  S.o = o;
  S.arnoldi_only = true;
  S.throttle = p->npts >= ((size_t)1 << 18);
  hp_status ret = HP_OK;
  hipError_t e = S.start((const cpx<double>*)v0, (cpx<double>*)x0.p, st);
  if (e == hipSuccess) e = S.advance(1 << 30, true);
  hp::KState ks;
  if (e == hipSuccess) e = hipMemcpyAsync(&ks, S.W->state.p, sizeof(ks), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) ret = from_hip(e);
  x0.release();
  if (ret != HP_OK) return ret;
  const int k = std::min(ks.iters, m);
  cpx<double>* h = (cpx<double>*)H;
  for (int i = 0; i <= m; ++i)
    for (int j = 0; j < m; ++j)
      h[(size_t)i * m + j] = (j < k && i <= j + 1) ? ks.Hraw[(size_t)j * (hp::kMaxRestart + 1) + i] : cpx<double>{0, 0};
  *steps = k;
  p->arnoldi_k = k;
  return S.inner_failed ? HP_E_NOT_CONVERGED : HP_OK;
}

hp_status hp_arnoldi_vector(hp_plan p, const void* y, int k, void* out, void* stream) {
  if (!p || !y || !out || k < 1 || k > p->arnoldi_k || !p->solver_ws_ptr) return HP_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  SolverWs* W = p->solver_ws_ptr;
  hp::KState* ks = (hp::KState*)W->state.p;
  hp::KrylovArgs K{};
  K.V = (cpx<double>*)W->V.p;
  K.npts = p->npts;
  K.vrs = (size_t)(W->restart + 1) * p->npts;
  K.state = ks;
  K.done = (int*)W->flags.p + W->nrhs;
  K.nrhs = 1;
  HP_TRY(hipMemcpyAsync(ks->y, y, (size_t)k * sizeof(cpx<double>), hipMemcpyHostToDevice, st));
  HP_TRY(hipMemcpyAsync(&ks->k, &k, sizeof(int), hipMemcpyHostToDevice, st));
  HP_TRY(hp::launch_fill_zero(K.done, sizeof(int), st));
  HP_TRY(hp::launch_lincomb(K, (cpx<double>*)out, p->npts, false, st));
  HP_TRY(hipStreamSynchronize(st));   // y and k are read from host memory
  return HP_OK;
}

hp_status hp_solve(hp_plan p, const void* f, void* x, int nrhs, const hp_solve_opts* opts, hp_solve_info* info,
                   void* stream) {
  if (!p || !f || !x || !opts || !info || nrhs < 0) return HP_E_INVALID;
  if (opts->restart < 1 || opts->restart > hp::kMaxRestart || opts->max_cycles < 1 || !(opts->rtol > 0) ||
      opts->side < HP_RIGHT || opts->side > HP_NONE)
    return HP_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  hp_status ret = HP_OK;
  for (int r0 = 0; r0 < nrhs; r0 += p->max_nrhs) {
    const int nr = std::min(p->max_nrhs, nrhs - r0);
    hp_status s = solve_batch(p, (const cpx<double>*)f + (size_t)r0 * p->npts, (cpx<double>*)x + (size_t)r0 * p->npts,
                              nr, *opts, info + r0, st);
    if (s != HP_OK && s != HP_E_NOT_CONVERGED && s != HP_E_NONFINITE) return s;
    if (s == HP_E_NONFINITE || (s == HP_E_NOT_CONVERGED && ret == HP_OK)) ret = s;
  }
  return ret;
}

hp_status hp_solver_create(hp_solver* out, hp_plan p, int nrhs, const hp_solve_opts* opts) {
  if (!out) return HP_E_INVALID;
  *out = nullptr;
  if (!p || !opts || nrhs < 1 || nrhs > p->max_nrhs) return HP_E_INVALID;
  if (opts->restart < 1 || opts->restart > hp::kMaxRestart || opts->max_cycles < 1 || !(opts->rtol > 0) ||
      opts->side < HP_RIGHT || opts->side > HP_NONE)
    return HP_E_INVALID;
  hp_solver_s* s = new (std::nothrow) hp_solver_s();
  if (!s) return HP_E_NOMEM;
  hipError_t e = s->ws.ensure(p->npts, p->fsize(), opts->restart, nrhs);
  if (e != hipSuccess) {
    s->ws.release();
    delete s;
    return from_hip(e);
  }
  s->sess.P = p;
  s->sess.W = &s->ws;
  s->sess.nrhs = nrhs;
  s->sess.o = *opts;
  s->sess.throttle = true;
  s->sess.use_graphs = p->npts * (size_t)nrhs < ((size_t)1 << 18) && step_graphs_enabled();
  *out = s;
  return HP_OK;
}

hp_status hp_solver_start(hp_solver s, const void* f, void* x, void* stream) {
  if (!s || !f || !x) return HP_E_INVALID;
  // a solve still in progress is abandoned: its enqueued work uses the same
  // workspace, so it has to drain first
  if (s->sess.phase != Session::kIdle && s->sess.phase != Session::kFinished && s->sess.st)
    HP_TRY(hipStreamSynchronize(s->sess.st));
  HP_TRY(s->sess.start((const cpx<double>*)f, (cpx<double>*)x, (hipStream_t)stream));
  return HP_OK;
}

hp_status hp_solver_advance(hp_solver s, int max_steps, int* finished) {
  if (!s || max_steps < 0 || s->sess.phase == Session::kIdle) return HP_E_INVALID;
  HP_TRY(s->sess.advance(max_steps, false));
  if (finished) *finished = s->sess.phase == Session::kFinished;
  return HP_OK;
}

hp_status hp_solver_advance_group(hp_solver* ss, int n, int max_steps, int* finished) {
  if (!ss || n < 1 || max_steps < 0) return HP_E_INVALID;
  for (int i = 0; i < n; ++i) {
    if (!ss[i] || ss[i]->sess.phase == Session::kIdle) return HP_E_INVALID;
    for (int k = 0; k < i; ++k)
      if (ss[k] == ss[i]) return HP_E_INVALID;
  }
  // the sessions of one stream form a group (several groups on several streams overlap)
  std::vector<hipStream_t> streams;
  std::vector<int> gidx(n);
  for (int i = 0; i < n; ++i) {
    size_t g = 0;
    while (g < streams.size() && streams[g] != ss[i]->sess.st) ++g;
    if (g == streams.size()) streams.push_back(ss[i]->sess.st);
    gidx[i] = (int)g;
  }
  std::vector<std::vector<hp::GroupMember>> grp(streams.size());
  std::vector<std::vector<Session*>> who(streams.size());
  for (int round = 0; round < max_steps; ++round) {
    for (size_t g = 0; g < streams.size(); ++g) {
      grp[g].clear();
      who[g].clear();
    }
    bool any = false;
    for (int i = 0; i < n; ++i) {
      Session& S = ss[i]->sess;
      hipError_t e;
      const Session::Poll r = S.poll(false, e);
      HP_TRY(e);
      if (r != Session::kPollStep) continue;
      any = true;
      hp::GroupMember m;
      if (S.group_member(&m)) {
        grp[gidx[i]].push_back(m);
        who[gidx[i]].push_back(&S);
      } else {
        HP_TRY(S.enqueue_step());   // a session the grouped kernels do not take steps alone
      }
    }
    for (size_t g = 0; g < streams.size(); ++g)
      for (size_t g0 = 0; g0 < grp[g].size(); g0 += hp::kMaxGroup) {
        const int cnt = (int)std::min(grp[g].size() - g0, (size_t)hp::kMaxGroup);
        if (cnt == 1) {
          HP_TRY(who[g][g0]->enqueue_step());   // alone: the same kernels as a group of one
          continue;
        }
        HP_TRY(hp::launch_group_step(&grp[g][g0], cnt, streams[g]));
        for (int q = 0; q < cnt; ++q) HP_TRY(who[g][g0 + q]->stepped_in_group());
      }
    if (!any) break;
  }
  // cycle transitions that became due after the last step
  for (int i = 0; i < n; ++i) {
    hipError_t e;
    (void)ss[i]->sess.poll(false, e);
    HP_TRY(e);
    if (finished) finished[i] = ss[i]->sess.phase == Session::kFinished;
  }
  return HP_OK;
}

hp_status hp_solver_wait(hp_solver s, hp_solve_info* info) {
  if (!s || !info || s->sess.phase == Session::kIdle) return HP_E_INVALID;
  HP_TRY(s->sess.advance(1 << 30, true));
  return s->sess.collect(info);
}

hp_status hp_solver_destroy(hp_solver s) {
  if (!s) return HP_E_INVALID;
  if (s->sess.st) (void)hipStreamSynchronize(s->sess.st);
  s->ws.release();
  delete s;
  return HP_OK;
}

hp_status hp_profile_apply(hp_plan p, const void* v, void* u, int nrhs, int reps, double* ms, double* bytes,
                           void* stream) {
  if (!p || !v || !u || !ms || !bytes || nrhs < 1 || nrhs > p->max_nrhs || reps < 1) return HP_E_INVALID;
  double acc[5];
  HP_TRY(time_passes(p, v, u, nrhs, reps, acc, (hipStream_t)stream));
  for (int i = 0; i < 5; ++i) ms[i] = acc[i];
  pass_bytes(p, nrhs, (int)p->fsize(), (int)p->fsize(), bytes);
  return HP_OK;
}

hp_status hp_plan_autotune(hp_plan p, double* before_ms, double* after_ms, void* stream) {
  if (!p) return HP_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  DevBuf v, u;
  HP_TRY(v.alloc(p->npts * p->fsize()));
  HP_TRY(u.alloc(p->npts * p->fsize()));
  HP_TRY(hp::launch_fill_zero(v.p, v.bytes, st));
  const int rk = p->real_kind();
  const int nl = p->n[p->dim - 1];
  const size_t S0 = p->npts / p->n[0];
  // per slot: candidate kind, line length, lines across, mode
  struct Slot { int kind, n, S, mode; bool used; };
  const Slot slots[5] = {{hp::kTuneRows, nl, 1, 0, true},
                         {hp::kTuneCols, p->n[1], p->n[2], 0, p->dim == 3},
                         {hp::kTuneCols, p->n[0], (int)S0, 1, true},
                         {hp::kTuneCols, p->n[1], p->n[2], 0, p->dim == 3},
                         {hp::kTuneCombine, nl, 1, 0, true}};
  // the fastest of three timings of every pass (the in-place 3-D passes run once per apply)
  auto measure = [&](double* t) -> hipError_t {
    for (int i = 0; i < 5; ++i) t[i] = INFINITY;
    for (int k = 0; k < 3; ++k) {
      double m[5];
      hipError_t e = time_passes(p, v.p, u.p, 1, 4, m, st);
      if (e != hipSuccess) return e;
      for (int i = 0; i < 5; ++i) t[i] = std::min(t[i], m[i]);
    }
    return hipSuccess;
  };
  double base[5];
  HP_TRY(measure(base));
  double best_t[5];
  for (int i = 0; i < 5; ++i) best_t[i] = base[i];
  // one pass at a time, the others at their current choice; a candidate must win by 2 %
  for (int sl = 0; sl < 5; ++sl) {
    if (!slots[sl].used) continue;
    hp::PassTune cand[64];
    const int nc = hp::tune_candidates(rk, slots[sl].kind, slots[sl].n, slots[sl].S, slots[sl].mode, p->K, cand, 64);
    hp::PassTune best = p->tune[sl];
    for (int c = 0; c < nc; ++c) {
      p->tune[sl] = cand[c];
      double t[5];
      HP_TRY(measure(t));
      if (t[sl] < 0.98 * best_t[sl]) {
        best_t[sl] = t[sl];
        best = cand[c];
      }
    }
    p->tune[sl] = best;
  }
  double fin[5];
  HP_TRY(measure(fin));
  HP_TRY(hipStreamSynchronize(st));
  if (before_ms) *before_ms = base[0] + base[1] + base[2] + base[3] + base[4];
  if (after_ms) *after_ms = fin[0] + fin[1] + fin[2] + fin[3] + fin[4];
  ++p->tune_gen;
  save_tune(*p);
  return HP_OK;
}

hp_status hp_plan_time_pass(hp_plan p, int slot) {
  if (!p || slot < -1 || slot > 4) return HP_E_INVALID;
  p->timer_slot = slot;
  p->timer_n = 0;
  return HP_OK;
}

hp_status hp_plan_pass_times(hp_plan p, double* ms, int cap, int* count) {
  if (!p || !count || cap < 0 || (cap > 0 && !ms)) return HP_E_INVALID;
  const size_t n = p->timer_n;
  p->timer_n = 0;
  for (size_t i = 0; i < n; ++i) {
    HP_TRY(hipEventSynchronize(p->timer_ev[2 * i + 1]));
    if ((int)i < cap) {
      float t = 0;
      HP_TRY(hipEventElapsedTime(&t, p->timer_ev[2 * i], p->timer_ev[2 * i + 1]));
      ms[i] = (double)t;
    }
  }
  *count = (int)n;
  return HP_OK;
}

hp_status hp_plan_destroy(hp_plan p) {
  if (!p) return HP_E_INVALID;
  (void)hipDeviceSynchronize();
  p->release_all();
  delete p;
  return HP_OK;
}

}  // extern "C"
