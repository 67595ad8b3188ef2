/*
 * helmpre — C ABI of the MI355X (gfx950) implementation of the interpolated
 * pseudodifferential preconditioner for the variable-media Helmholtz equation
 *     c^2 Lap u + omega^2 u + i omega a u = f            (Eqn. 001)
 * of Acosta, Khajah and Palacios (arXiv 2409.16172), together with the
 * finite-difference operator P_N it preconditions and a restarted GMRES solver.
 *
 * Conventions shared by every entry point
 *   - Grids: d = 2 or 3 dimensions, n[j] points per axis, each a power of two in
 *     [8, 2048] (FP64 plans) or [8, 4096] (mixed plans), or an even product of
 *     2, 3 and 5 in [8, 4800] (such as the N = 180 * 2^k and 2400 of Section 5.1;
 *     these lines are transformed in LDS by mixed-radix stages), fewer than 2^32
 *     points in all; side len[j]; spacing h_j = len[j]/n[j]; periodic boundary
 *     conditions (Section 5).
 *   - Fields: row-major with the last axis contiguous, complex interleaved
 *     (re, im); several right-hand sides are stored one after another
 *     ("batch outermost": [nrhs][n0][n1]([n2])).
 *   - Host arrays (media, options) are read during the call and copied; the
 *     library never keeps a host pointer.  Device arrays are HIP device memory
 *     owned by the caller.
 *   - `stream` is a hipStream_t (NULL = the default stream).  apply and matvec
 *     only enqueue work; they allocate nothing and return before it completes.
 *   - Errors are status codes; argument and media errors are detected before
 *     anything is enqueued.  No C++ exception crosses this interface.
 *   - A plan is not re-entrant: calls on one plan must not overlap (they share
 *     the plan's workspace).  Distinct plans are independent.
 */
#ifndef HELMPRE_H
#define HELMPRE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hp_plan_s* hp_plan;

typedef enum {
  HP_OK = 0,
  HP_E_INVALID = 1,        /* bad argument or option                                 */
  HP_E_SHAPE = 2,          /* grid size not supported                                 */
  HP_E_MEDIA = 3,          /* media not finite / not positive, or a zero symbol denominator */
  HP_E_LAYER = 4,          /* c differs from the background c0 where zeta > 0        */
  HP_E_NONFINITE = 5,      /* non-finite right-hand side or residual (that one stops)  */
  HP_E_DEVICE = 6,         /* a HIP call failed                                       */
  HP_E_NOMEM = 7,          /* device allocation failed                                */
  HP_E_NOT_CONVERGED = 8   /* solve stopped at max_cycles above the tolerance         */
} hp_status;

typedef enum { HP_FP64 = 0, HP_MIXED = 1 } hp_precision;
typedef enum { HP_SYMBOL_CONTINUOUS = 0, HP_SYMBOL_DISCRETE = 1 } hp_symbol;

typedef struct {
  int dim;          /* 2 or 3                                        */
  int n[3];         /* points per axis (n[2] ignored when dim = 2)  */
  double len[3];    /* side lengths                                  */
} hp_grid;

/* Absorbing layer by a complex wave speed gamma = c (1 - i zeta)
 * (Eqn. Complex_wave_speed).  The medium must satisfy c = c0 wherever
 * zeta > 0 (Section 4.4); zeta >= 0 on the host, n[0]*...*n[d-1] values. */
typedef struct {
  const double* zeta;   /* host, may be NULL (no layer)        */
  double c0;            /* background speed c_o (> 0)          */
} hp_layer;

/* Preconditioner options.
 *   m_real     M: real-axis interpolation nodes (Section 4.1).  1 gives the
 *              one-node preconditioner Q_1 of Eqn. OneInterpPoint (node c0,
 *              no layer nodes).  With a layer c0 is always a node and M >= 3.
 *   m_layer    M~: layer nodes zeta_1..zeta_M~ (Section 4.4), >= 1 when a layer is given.
 *   nodes_real optional explicit increasing real nodes (host, m_real values)
 *   nodes_zeta optional explicit increasing layer nodes (host, m_layer values > 0)
 *   a_nodes    optional damping a(c_m) at the real nodes (host, m_real values)
 *   a_floor    lower bound on the symbol damping of every node whose speed
 *              is real (Im gamma_n = 0: the real-axis nodes, and the bivariate
 *              and layer-tensor nodes with zero imaginary part), where a = 0
 *              would put zeros of the symbol denominator on the grid (Section
 *              3 assumes a_min > 0).  Nodes with Im gamma_n < 0 (layer nodes)
 *              keep the damping of c0 unfloored.  The operator P_N keeps the
 *              true a.  0 disables it
 *   symbol     HP_SYMBOL_CONTINUOUS: |xi|^2 as in Eqn. 021;
 *              HP_SYMBOL_DISCRETE: the 5/7-point stencil's own symbol
 *   precision  HP_FP64, or HP_MIXED (FFTs, symbol multiply, combine and the
 *              Arnoldi stencil in FP32; orthogonalisation, least squares, true
 *              residual and set-up in FP64)
 *   max_nrhs   largest batch one apply/matvec call processes at once (>= 1);
 *              larger batches are processed in chunks
 *   interp_order  real-axis interpolation: 0 or 1 piecewise linear (Section
 *              4.1), 2 or 3 piecewise Lagrange of that degree through
 *              consecutive nodes (the other polynomial bases of Sections 1
 *              and 4.3; capped at M - 1); the layer leg stays linear
 *   m_damp     0 or 1: the damping enters the symbol through one value per real
 *              node (a as a function of c, Section 4); >= 2: bivariate
 *              interpolation in (c, a), the extension the concluding remarks
 *              name for a damping independent of c: m_damp equidistant damping
 *              nodes on [a_min, a_max], node (c_m, a_r) for every pair (K =
 *              M m_damp <= 64), tensor-product hat weights.  Needs no layer
 *              and interp_order <= 1 (else HP_E_INVALID); a uniform a falls
 *              back to the univariate scheme
 *   layer_tensor  with a layer: replace the two legs of Eqn. 405 by a tensor grid
 *              of M speed nodes (equidistant on [c_min, c_max]) by m_layer + 1
 *              nodes of Im gamma = -c zeta (equidistant on [-max c zeta, 0]),
 *              node gamma = c_m + i g_r (K = M (m_layer + 1) <= 64), tensor-product
 *              hat weights in (Re gamma, Im gamma): c need not equal c0 inside
 *              the layer (no HP_E_LAYER).  Needs interp_order <= 1 and no m_damp
 *              (else HP_E_INVALID); ignored without a layer                     */
typedef struct {
  int m_real;
  int m_layer;
  const double* nodes_real;
  const double* nodes_zeta;
  const double* a_nodes;
  double a_floor;
  int symbol;
  int precision;
  int max_nrhs;
  int interp_order;
  int m_damp;
  int layer_tensor;
} hp_plan_opts;

/* Restarted GMRES(restart) on P_N x = f, starting from the x passed in.
 *   side HP_RIGHT (default, 0): P_N Q y = f, x = Q y; stops when the FP64 true
 *        residual ||f - P_N x||_2 <= rtol ||f||_2 at a restart.
 *   side HP_LEFT: Q P_N x = Q f (Eqn. MainDiscretePrecond as written); stops when
 *        the preconditioned residual ||Q (f - P_N x)|| <= rtol ||Q f|| at a restart.
 *   side HP_NONE: plain GMRES on P_N x = f (FP64), the unpreconditioned
 *        reference of the GMRES comparison of Section 5.1.
 * Every side stops after max_cycles cycles. */
enum { HP_RIGHT = 0, HP_LEFT = 1, HP_NONE = 2 };
/* Operators of hp_arnoldi only (spectral diagnostics): (Q P_N)^{-1} and P_N^{-1}, each
 * application an inner restarted GMRES(64) solve to 1e-10 relative residual (Q P_N x = v
 * with v as the given right-hand side; P_N x = v preconditioned on the right). */
enum { HP_LEFT_INVERSE = 3, HP_NONE_INVERSE = 4 };
typedef struct {
  int restart;       /* 1..64                 */
  int max_cycles;    /* >= 1                  */
  double rtol;       /* > 0                   */
  int side;          /* HP_RIGHT, HP_LEFT, HP_NONE */
} hp_solve_opts;

typedef struct {
  int iters;                 /* Arnoldi steps taken                                  */
  int cycles;                /* restart cycles run                                   */
  double rel_true_residual;  /* ||f - P_N x|| / ||f|| at return (FP64)               */
  int status;                /* HP_OK or HP_E_NOT_CONVERGED                          */
  double rel_prec_residual;  /* the residual the stopping test used: the true one for
                                HP_RIGHT and HP_NONE, ||Q(f - P_N x)|| / ||Q f|| for
                                HP_LEFT                                              */
} hp_solve_info;

/* Read-only description of a plan (for tests and reports). */
typedef struct {
  int dim, n[3];
  int K, M, Mt, mo;          /* node fields, real nodes, layer nodes, index of c0 */
  double cmin, cmax, zeta_max;
  double cnode[64];          /* real nodes                  */
  double znode[65];          /* zeta_0 = 0, zeta_1..zeta_Mt */
  double ahat[64];           /* symbol damping per node     */
  double gamma_re[64], gamma_im[64];  /* node speeds gamma_n (K) */
  size_t workspace_bytes;    /* device bytes held by the plan for apply/matvec */
  int precision;
  int interp_order;          /* real-axis interpolation degree in effect */
  int m_damp;                /* damping nodes of the bivariate scheme (0: univariate);
                                real node (c_m, a_r) is node m + M r */
  double anode[64];          /* damping nodes a_r (bivariate), or the Im gamma nodes
                                g_r (layer tensor; node gamma = c_m + i g_r) */
  int tune[5][4];            /* run-time choices of passes A, A', B, M, C: threads per
                                line, lines per workgroup, radix schedule, node groups
                                (0 = built-in); see hp_plan_autotune */
  int layer_tensor;          /* 1: the layer tensor is in use */
} hp_plan_info;

/* Build a plan: upload and validate the media, place the nodes, and compute in
 * FP64 on the device the per-point interpolation records, the stencil
 * coefficients, the symbol tables and the node masks (Section 4, Eqn. 021,
 * 403/405; Section 5).  Blocks until the plan is ready.
 *   c      host, wave speed > 0 at every point
 *   a      host damping >= 0 at every point, or NULL (a = 0)
 *   layer  NULL: no absorbing layer
 * Errors: HP_E_INVALID, HP_E_SHAPE, HP_E_MEDIA (non-finite or non-positive
 * media, or a symbol denominator that vanishes on the grid), HP_E_LAYER,
 * HP_E_NOMEM, HP_E_DEVICE.  On error *out is NULL. */
hp_status hp_plan_create(hp_plan* out, const hp_grid* grid, double omega, const double* c,
                         const double* a, const hp_layer* layer, const hp_plan_opts* opts,
                         void* stream);

/* Device bytes a plan with these options holds for apply/matvec (excluding the
 * solver's Krylov storage), and the solver's extra bytes for nrhs and restart. */
size_t hp_plan_workspace_bytes(const hp_grid* grid, const hp_plan_opts* opts, int K);
size_t hp_solve_workspace_bytes(const hp_grid* grid, int restart, int nrhs);

hp_status hp_plan_query(hp_plan p, hp_plan_info* info);

/* u = Q_M v (Eqn. 403): one forward FFT of each field, K symbol multiplies and
 * inverse FFTs, and the pointwise combine with the piecewise-linear weights of
 * the local complex speed.  v, u: device, nrhs fields, complex128 for FP64
 * plans and complex64 for mixed plans.  u == v is allowed.  Any nrhs >= 0: the
 * fields run in batches of at most the plan's max_nrhs, one after another. */
hp_status hp_apply_precond(hp_plan p, const void* v, void* u, int nrhs, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): u = Q_M v exactly as
 * hp_apply_precond computes it (same kernels, bitwise the same result), but with
 * the intermediate spectrum and the K node fields in a static device array of
 * HP_STATIC_SCRATCH_BYTES that the library holds on every GPU it runs on until
 * the process ends, instead of the plan's workspace.  Calls no hipMalloc,
 * hipFree or other allocating routine.  One field needs (1 + K) N^d S bytes of it
 * (S = 16 for FP64 plans, 8 for mixed), rounded up to 256 between the two parts;
 * a batch runs in chunks of as many fields as fit.  Returns HP_E_INVALID, with
 * the sizes in hp_last_error(), when one field does not fit.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads, other plans) race and must be serialised by the caller.
 * Nothing needs clearing between calls: every part of the array a call reads
 * was written earlier in the same call. */
#define HP_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
hp_status hp_apply_precond_static(hp_plan p, const void* v, void* u, int nrhs, void* stream);

/* y = P_N u: second-order centred differences of Eqn. 003 with periodic
 * boundaries, gamma^2 in place of c^2 (Section 4.4, Section 5).  Same dtypes as
 * apply.  y must not alias u. */
hp_status hp_matvec(hp_plan p, const void* u, void* y, int nrhs, void* stream);

/* Restarted GMRES on P_N x = f with right preconditioner Q_M (the left form of
 * Eqn. MainDiscretePrecond rearranged so that the residual GMRES minimises is
 * the true one).  f, x: device complex128 [nrhs][N^d] whatever the plan
 * precision; x holds the initial guess on entry and the solution on return.
 * info: host array of nrhs entries.  Blocks until every right-hand side has
 * converged or max_cycles is reached.  Krylov storage is allocated on first
 * use and kept by the plan.  Returns HP_E_NOT_CONVERGED if any right-hand side
 * stopped above rtol, HP_E_NONFINITE if any had a non-finite norm or residual
 * (that one stops where the value is found: a non-finite f or initial residual
 * leaves x as it was; a residual that turns non-finite during the solve stops
 * it at that restart, x holding the update made so far, and its residuals are
 * reported as NaN; the others are solved); x and info are
 * filled in either case, info[r].status giving each right-hand side's outcome.
 * With the environment variable HP_STEP_GRAPHS=1, grids of fewer than 2^18 points
 * (times nrhs) run each Arnoldi step as a HIP graph captured once per step index
 * and solver configuration (also in hp_solver sessions); results are bitwise those
 * of the direct launches. */
hp_status hp_solve(hp_plan p, const void* f, void* x, int nrhs, const hp_solve_opts* opts,
                   hp_solve_info* info, void* stream);

/* Spectral diagnostics: the two ends of the spectrum that define the condition
 * numbers of Eqn. Cond (Section 5).
 *
 * hp_arnoldi: m Arnoldi steps (1..64) of the operator P_N Q (HP_RIGHT), Q P_N (HP_LEFT),
 * P_N (HP_NONE), (Q P_N)^{-1} (HP_LEFT_INVERSE) or P_N^{-1} (HP_NONE_INVERSE) from v0
 * (device complex128, N^d; normalised first, no preconditioner applied to it), in FP64
 * with the orthogonalisation of hp_solve (classical Gram-Schmidt with a second
 * projection); the preconditioner runs at the plan's precision.  Returns
 * HP_E_NOT_CONVERGED (H filled in) if an inner solve of an inverse operator stopped
 * above its tolerance.
 * H: host array (m+1) x m complex128, row-major, receives the upper Hessenberg matrix
 * with A V_k = V_{k+1} H[:k+1, :k]; *steps = k (fewer than m only on an invariant
 * subspace; 0 for v0 = 0).  The basis V_k stays in the plan's solver workspace until the
 * next hp_arnoldi or hp_solve on the plan.  Allocates a temporary device vector; blocks. */
hp_status hp_arnoldi(hp_plan p, const void* v0, int m, int side, void* H, int* steps, void* stream);

/* out = V_k y (device complex128, N^d) from the basis the last hp_arnoldi on this plan
 * left (y: host, k complex128, 1 <= k <= its steps): a Ritz vector, or the start of a
 * restarted run.  HP_E_INVALID if no such basis is held.  Blocks. */
hp_status hp_arnoldi_vector(hp_plan p, const void* y, int k, void* out, void* stream);

/* Ritz pairs of the k x k leading block H_k of an Arnoldi Hessenberg matrix H (host,
 * (m+1) x m complex128 row-major as hp_arnoldi returns it, 1 <= k <= m <= 64).
 * harmonic = 0: the Ritz values eig(H_k), which approach the eigenvalues of largest
 * modulus; harmonic = 1: the harmonic Ritz values eig(H_k + |h_{k+1,k}|^2 H_k^{-H} e_k
 * e_k^T), which approach those nearest zero.  theta: host k complex128, unordered.
 * Y (host k x k complex128, row i = unit vector y_i of theta_i) and resid (host k
 * doubles, ||A V_k y_i - theta_i V_k y_i|| for the orthonormal basis) may be NULL.
 * Host only (no device work).  Errors: HP_E_INVALID (bad sizes; H_k singular for
 * harmonic = 1), HP_E_NONFINITE, HP_E_NOT_CONVERGED (the QR iteration did not deflate). */
hp_status hp_ritz_values(const void* H, int m, int k, int harmonic, void* theta, void* Y, double* resid);

/* One end of the spectrum of the operator of `side` (HP_RIGHT, HP_LEFT, HP_NONE): the
 * eigenvalue of largest (smallest = 0) or smallest (smallest = 1) modulus, by explicitly
 * restarted Arnoldi runs of m steps (2..64) from v0 (device complex128, N^d), each
 * restarted from the wanted Ritz vector, until its residual relative to the Ritz value
 * is <= tol or after max_restarts restarts.  The smallest end is the largest Ritz value
 * of the inverse operator (HP_LEFT_INVERSE for HP_LEFT and HP_RIGHT, whose operators are
 * similar; HP_NONE_INVERSE for HP_NONE), inverted.  lambda: host complex128;
 * *rel_resid: that relative residual (of the inverse operator's pair for the smallest
 * end); *runs: Arnoldi runs made.  Returns HP_E_NOT_CONVERGED (with the last estimate
 * filled in) if tol was not reached or an inner solve stopped above its tolerance.
 * Uses the plan's solver workspaces; allocates a temporary device vector; blocks. */
hp_status hp_extreme_eigenvalue(hp_plan p, const void* v0, int m, int side, int smallest, int max_restarts,
                                double tol, void* lambda, double* rel_resid, int* runs, void* stream);

/* Resumable solves, for callers that interleave several solves (a serving
 * loop).  A solver owns the Krylov workspace of nrhs right-hand sides
 * (hp_solve_workspace_bytes) and runs the same right-preconditioned restarted
 * GMRES as hp_solve on one stream, with its state kept on the device.
 *   hp_solver_create   allocate the workspace (nrhs <= the plan's max_nrhs)
 *   hp_solver_start    enqueue the start of a solve of f (x: initial guess,
 *                      overwritten by the solution); f, x stay owned by the
 *                      caller and must remain valid until the solve finishes.
 *                      A solve still in progress on the solver is abandoned
 *                      (its enqueued work is waited for first).
 *   (hp_solver_advance and hp_solver_wait before any start: HP_E_INVALID.)
 *   hp_solver_advance  enqueue at most max_steps further Arnoldi steps without
 *                      waiting for the device; *finished = 1 once the solve
 *                      has ended (converged or max_cycles)
 *   hp_solver_wait     block until the solve ends; fills info[nrhs]; returns
 *                      HP_E_NOT_CONVERGED if a right-hand side stopped above rtol,
 *                      HP_E_NONFINITE if one met a non-finite norm or residual
 *                      (as hp_solve; info[r].status tells which)
 * A plan's preconditioner workspace is shared by everything that runs on it:
 * solvers of one plan must not progress concurrently on different streams. */
typedef struct hp_solver_s* hp_solver;
hp_status hp_solver_create(hp_solver* out, hp_plan p, int nrhs, const hp_solve_opts* opts);
hp_status hp_solver_start(hp_solver s, const void* f, void* x, void* stream);
hp_status hp_solver_advance(hp_solver s, int max_steps, int* finished);
/* Batching of several solves (different grids, media and frequencies) into shared
 * launches: like hp_solver_advance for each of the n distinct solvers s[0..n-1],
 * without waiting for the device, but every round takes the next Arnoldi step of all
 * of them that are ready for one, and the steps of the solvers the grouped kernels
 * take run as one launch per pass over all of them (passes A, A', B, M, C of Q_M in
 * Eqn. 403, the Gram-Schmidt sweep with the stencil P_N, the least-squares update and
 * the basis update; at most 8 per launch).  Those are: one right-hand side, right
 * preconditioning (HP_RIGHT), a mixed-precision plan, grids of at most 2^21 points
 * with power-of-two lines of 256-1024 points (2-D) or 128-512 (3-D), restart <= 32,
 * the combine's built-in workgroup shape (single solves of such sessions run the same
 * kernels as a group of one).  The others step with their own launches in the same
 * rounds.  The solvers started on one stream form one group, launched on that stream;
 * groups on different streams overlap on the device.  Results are bitwise those of
 * hp_solver_advance.  HP_E_INVALID for a solver not started or listed twice.
 * finished: n entries (may be NULL), 1 where the solve has ended. */
hp_status hp_solver_advance_group(hp_solver* s, int n, int max_steps, int* finished);
hp_status hp_solver_wait(hp_solver s, hp_solve_info* info);
hp_status hp_solver_destroy(hp_solver s);

/* Diagnostic timing of the preconditioner passes (for benchmarks): computes
 * u = Q_M v (as hp_apply_precond, nrhs <= max_nrhs), then launches each
 * out-of-place pass `reps` times back to back between two HIP events on
 * `stream` (the in-place 3-D middle-axis passes once).  u holds Q_M v on
 * return.  Blocks until done.  ms[5] receives the average milliseconds per
 * launch of the passes in order
 *   0: forward transform along the last (contiguous) axis
 *   1: forward transform along the middle axis (3-D only, else 0)
 *   2: forward transform along axis 0, symbol multiplies and inverse transforms
 *   3: inverse transform along the middle axis of the K fields (3-D only, else 0)
 *   4: inverse transform along the last axis and interpolation combine
 * bytes[5] receives the algorithmic HBM bytes of each pass per launch: the
 * fields each pass must read and write, counting only the node fields that
 * some point of a row uses (the others are neither written nor read). */
hp_status hp_profile_apply(hp_plan p, const void* v, void* u, int nrhs, int reps, double* ms, double* bytes,
                           void* stream);

/* Pass timer (for benchmarks): hp_plan_time_pass(p, slot) makes every later
 * launch of pass `slot` (numbered as in hp_profile_apply; -1 switches the timer
 * off) on this plan, in applies, solves and solver sessions alike, carry a pair of
 * HIP events that take the kernel's own start and end times on the launch's
 * stream (hipExtLaunchKernelGGL: no extra packets, so the timed work is not
 * changed), and clears the record.
 * Launches captured into a graph and launches beyond 65536 per read are not
 * timed.  hp_plan_pass_times waits for the recorded launches, stores the
 * milliseconds of each in launch order in ms[0..min(count, cap)-1], sets *count
 * to the number recorded and clears the record.  A launch whose right-hand sides
 * had all stopped returns at once and is recorded too (a few microseconds).  The
 * events are created on demand and kept until hp_plan_destroy. */
hp_status hp_plan_time_pass(hp_plan p, int slot);
hp_status hp_plan_pass_times(hp_plan p, double* ms, int cap, int* count);

/* Autotuner of the transform passes: for each pass in turn, times the plan's apply
 * (one right-hand side) under every valid run-time choice — threads per line, lines
 * per workgroup and radix schedule of the mixed-radix passes (N = 2^a 3^b 5^c),
 * node groups per column tile of the power-of-two symbol pass, node splits of the
 * power-of-two combine (lines of at most 1024 points) — and keeps the fastest (by
 * at least 2 %); the plan then uses it for every apply, solve step and session.
 * Only the radix schedule and the node splits change results (rounding).
 * If the environment variable HP_TUNE_CACHE names a file the choices are appended
 * to it, and hp_plan_create reads it for plans of the same grid, precision and K.
 * before_ms / after_ms (may be NULL): the summed per-pass apply time before and
 * after.  Allocates two temporary device fields; blocks (a few hundred applies). */
hp_status hp_plan_autotune(hp_plan p, double* before_ms, double* after_ms, void* stream);

hp_status hp_plan_destroy(hp_plan p);

const char* hp_status_str(hp_status st);

/* Description of the last HIP failure on this thread (function, source line and
 * the runtime's message), or "" if none. */
const char* hp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HELMPRE_H */
