/*
 * CPU FP64 oracle for the interpolated pseudodifferential Helmholtz
 * preconditioner (Acosta, Khajah, Palacios, arXiv 2409.16172).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * Everything here is written for a reader to check against the paper by eye:
 *   - the discrete Fourier transform by an iterative radix-2 Cooley-Tukey FFT
 *     (and a naive O(N^2) DFT used to pin it);
 *   - the second-order centred finite-difference operator P_N with periodic
 *     boundary conditions (Section 5, operator of Eqn. 003 with c replaced by
 *     the complex speed gamma of Eqn. Complex_wave_speed);
 *   - the interpolated preconditioner Q_M of Eqn. 403/405 evaluated as one
 *     forward transform, K symbol multiplies, K inverse transforms and the
 *     hat-weighted sum (Section 4.1, "Algorithm"), with the principal symbol
 *     q_{-2} of Eqn. 021;
 *   - the exact pseudodifferential operator Q of Eqn. Precond by brute force;
 *   - textbook restarted GMRES(m) with modified Gram-Schmidt and Givens
 *     rotations (Saad and Schultz 1986), right or left preconditioned.
 *
 * Readings of points the paper leaves open are listed in the design notes and
 * restated where they are used.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cx;

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define OR_OK 0
#define OR_E_INVALID 1
#define OR_E_SHAPE 2
#define OR_E_MEDIA 3
#define OR_E_LAYER 4
#define OR_E_NOMEM 7
#define OR_E_NOT_CONVERGED 8

/* ------------------------------------------------------------------ */
/* Problem description (mirrors what the preconditioner needs).       */
/* ------------------------------------------------------------------ */
typedef struct {
    int dim;
    int n[3];
    double len[3];
    double omega;
    const double* c;      /* real wave speed, N^d                         */
    const double* a;      /* damping, N^d (NULL = 0)                      */
    const double* zeta;   /* layer profile >= 0, N^d (NULL = no layer)    */
    double c0;            /* background speed c_o                          */
    int m_real;           /* M  (real-axis nodes)                          */
    int m_layer;          /* M~ (layer nodes)                              */
    int symbol;           /* 0: |xi|^2 (Eqn. 021), 1: stencil symbol       */
    double a_floor;       /* floor on the symbol damping of real nodes     */
    const double* nodes_real;  /* optional explicit real nodes (length m_real)  */
    const double* nodes_zeta;  /* optional explicit zeta nodes (length m_layer) */
    const double* a_nodes;     /* optional damping at the real nodes            */
    int interp_order;          /* real-axis interpolation: 1 (or 0) piecewise linear, 2 or 3
                                  piecewise Lagrange of that degree                */
    int m_damp;                /* >= 2: bivariate interpolation in (c, a) with m_damp
                                  equidistant damping nodes on [a_min, a_max]; 0/1: a is
                                  treated as a function of c (one damping per real node) */
    int layer_tensor;          /* 1: with a layer, interpolate on the tensor grid of
                                  (Re gamma, Im gamma) nodes instead of the two legs of
                                  Eqn. 405, so that c need not equal c_o in the layer  */
} or_problem;

/* Derived quantities of the preconditioner (filled by or_setup). */
typedef struct {
    int M;            /* real nodes actually used          */
    int Mt;           /* layer nodes actually used (0 if no layer) */
    int K;            /* M + Mt                            */
    int mo;           /* index of c_o among real nodes (-1 if not needed) */
    double cmin, cmax, zmax;
    double cnode[64];      /* real nodes c_1..c_M             */
    double znode[65];      /* zeta_0 = 0, zeta_1..zeta_Mt     */
    double ahat[64];       /* symbol damping per node (K)     */
    double gre[64], gim[64]; /* gamma_n per node (K)          */
    int order;             /* real-axis interpolation degree (1, 2 or 3) */
    int Ma;                /* second-axis nodes of a tensor scheme (0: none) */
    double anode[64];      /* a_1..a_Ma (bivariate in (c, a)) or the Im gamma nodes
                              (layer tensor); node (m, r) is node m + M r */
    double amin, amax;
    int tensor;            /* 1: the second axis is Im gamma (layer tensor) */
} or_setup_t;

static long npoints(const or_problem* p) {
    long n = 1;
    for (int d = 0; d < p->dim; ++d) n *= p->n[d];
    return n;
}

/* ------------------------------------------------------------------ */
/* Fourier transforms.                                                 */
/* Forward: X(k) = sum_j x(j) exp(-2 pi i j k / n)   (unnormalised)    */
/* Inverse: x(j) = sum_k X(k) exp(+2 pi i j k / n)   (caller divides)  */
/* The sign follows the Fourier transform of Eqn. FT.                  */
/* ------------------------------------------------------------------ */
void or_dft1d_naive(int n, const cx* x, cx* y, int sign) {
    for (int k = 0; k < n; ++k) {
        cx s = 0;
        for (int j = 0; j < n; ++j) {
            long m = ((long)j * k) % n;
            double ang = sign * 2.0 * M_PI * (double)m / (double)n;
            s += x[j] * (cos(ang) + I * sin(ang));
        }
        y[k] = s;
    }
}

static int is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

/* In-place iterative radix-2 decimation-in-time FFT.  `w` holds
 * exp(sign 2 pi i m / n) for m < n/2, each entry computed directly. */
static void fft1d_tab(int n, cx* x, const cx* w) {
    for (int i = 1, j = 0; i < n; ++i) {           /* bit-reversal permutation */
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cx t = x[i]; x[i] = x[j]; x[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {        /* butterflies of size len */
        int half = len >> 1, stride = n / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < half; ++k) {
                cx u = x[i + k];
                cx v = x[i + k + half] * w[k * stride];
                x[i + k] = u + v;
                x[i + k + half] = u - v;
            }
    }
}

static cx* twiddles(int n, int sign) {
    cx* w = (cx*)malloc(sizeof(cx) * (size_t)(n / 2 + 1));
    if (!w) return NULL;
    for (int m = 0; m < n / 2 + 1; ++m) {
        double ang = sign * 2.0 * M_PI * (double)m / (double)n;
        w[m] = cos(ang) + I * sin(ang);
    }
    return w;
}

/* Lengths that are not powers of two (the grids N = 180 * 2^k etc. of Example 1,
 * Section 5.1): recursive decimation in time on the smallest prime factor p of n.
 * With m = n/p and X_r the m-point transform of x[r], x[r+p], x[r+2p], ...,
 *     X[k + q m] = sum_{r<p} exp(sign 2 pi i r (k + q m) / n) X_r[k],
 * for k < m, q < p.  `w` holds exp(sign 2 pi i j / ntop) for j < ntop, and a
 * sub-transform of length n reads it with step ntop/n. */
static int smallest_factor(int n) {
    for (int f = 2; f * f <= n; ++f) if (n % f == 0) return f;
    return n;
}

static int fft_mixed(int n, const cx* in, long is, cx* out, const cx* w, int ntop) {
    if (n == 1) { out[0] = in[0]; return OR_OK; }
    int p = smallest_factor(n), m = n / p;
    for (int r = 0; r < p; ++r) {
        int rc = fft_mixed(m, in + (long)r * is, is * p, out + (long)r * m, w, ntop);
        if (rc) return rc;
    }
    cx* tmp = (cx*)malloc(sizeof(cx) * (size_t)n);
    if (!tmp) return OR_E_NOMEM;
    long step = ntop / n;
    for (int k = 0; k < m; ++k)
        for (int q = 0; q < p; ++q) {
            cx acc = 0;
            for (int r = 0; r < p; ++r) acc += w[(((long)r * (k + (long)q * m)) % n) * step] * out[(long)r * m + k];
            tmp[k + (long)q * m] = acc;
        }
    memcpy(out, tmp, sizeof(cx) * (size_t)n);
    free(tmp);
    return OR_OK;
}

/* One line of length n in place: radix-2 for powers of two, else mixed radix. */
static int fft_line(int n, cx* x, int sign) {
    if (is_pow2(n)) {
        cx* w = twiddles(n, sign);
        if (!w) return OR_E_NOMEM;
        fft1d_tab(n, x, w);
        free(w);
        return OR_OK;
    }
    cx* w = (cx*)malloc(sizeof(cx) * (size_t)n);
    cx* y = (cx*)malloc(sizeof(cx) * (size_t)n);
    if (!w || !y) { free(w); free(y); return OR_E_NOMEM; }
    for (int j = 0; j < n; ++j) {
        double ang = sign * 2.0 * M_PI * (double)j / (double)n;
        w[j] = cos(ang) + I * sin(ang);
    }
    int rc = fft_mixed(n, x, 1, y, w, n);
    if (!rc) memcpy(x, y, sizeof(cx) * (size_t)n);
    free(w);
    free(y);
    return rc;
}

int or_fft1d(int n, cx* x, int sign) {
    if (n < 1) return OR_E_SHAPE;
    return fft_line(n, x, sign);
}

/* d-dimensional transform, one axis at a time.  inverse != 0 applies the
 * 1/N^d factor so that the inverse undoes the forward transform. */
int or_fftnd(int dim, const int* n, cx* x, int inverse) {
    long tot = 1;
    for (int d = 0; d < dim; ++d) { if (n[d] < 1) return OR_E_SHAPE; tot *= n[d]; }
    int sign = inverse ? +1 : -1;
    for (int ax = 0; ax < dim; ++ax) {
        int len = n[ax];
        long stride = 1;
        for (int d = ax + 1; d < dim; ++d) stride *= n[d];
        long outer = tot / (stride * len);
        long nlines = outer * stride;
        int err = OR_OK;
        /* the lines are independent (OpenMP builds take them in parallel) */
#ifdef _OPENMP
#pragma omp parallel
#endif
        {
            cx* line = (cx*)malloc(sizeof(cx) * (size_t)len);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (long q = 0; q < nlines; ++q) {
                long o = q / stride, s = q % stride;
                cx* base = x + o * stride * len + s;
                int rc = line ? OR_OK : OR_E_NOMEM;
                if (rc == OR_OK) {
                    for (int i = 0; i < len; ++i) line[i] = base[(long)i * stride];
                    rc = fft_line(len, line, sign);
                    for (int i = 0; i < len; ++i) base[(long)i * stride] = line[i];
                }
                if (rc) {
#ifdef _OPENMP
#pragma omp critical
#endif
                    err = rc;
                }
            }
            free(line);
        }
        if (err) return err;
    }
    if (inverse) {
        double sc = 1.0 / (double)tot;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (long i = 0; i < tot; ++i) x[i] *= sc;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Interpolation nodes (Section 4.1 and Section 4.4).                  */
/* ------------------------------------------------------------------ */

/* Real nodes: c_1 = c_min < ... < c_M = c_max.  Without a layer they are
 * equidistant (the setting of Lemma 3).  With a layer c_o must be a node
 * (Section 4.4); the reading used here splits the nodes into two equidistant
 * runs on [c_min, c_o] and [c_o, c_max], with s = round-half-down of
 * (c_o - c_min)/(c_max - c_min) * (M - 1) intervals below c_o, kept in
 * [1, M-2] when c_o is strictly inside (M is raised to 3 if needed).
 * A homogeneous medium (c_max = c_min) or M = 1 gives the single node c_o
 * (the one-node preconditioner Q_1 of Eqn. OneInterpPoint). */
static int real_nodes(const or_problem* p, or_setup_t* s, int has_layer) {
    int M = p->m_real;
    if (M < 1 || M > 64) return OR_E_INVALID;
    if (p->nodes_real) {
        for (int i = 0; i < M; ++i) {
            s->cnode[i] = p->nodes_real[i];
            if (!(s->cnode[i] > 0.0)) return OR_E_INVALID;
            if (i > 0 && !(s->cnode[i] > s->cnode[i - 1])) return OR_E_INVALID;
        }
        s->M = M;
        s->mo = -1;
        for (int i = 0; i < M; ++i) if (s->cnode[i] == p->c0) s->mo = i;
        if (has_layer && s->mo < 0) return OR_E_LAYER;
        return OR_OK;
    }
    double lo = s->cmin, hi = s->cmax, co = p->c0;
    if (M == 1 || !(hi > lo)) {
        s->M = 1;
        s->cnode[0] = (M == 1) ? co : lo;
        s->mo = (s->cnode[0] == co) ? 0 : -1;
        if (has_layer && s->mo < 0) return OR_E_LAYER;
        return OR_OK;
    }
    if (!has_layer) {
        for (int i = 0; i < M; ++i) s->cnode[i] = lo + (hi - lo) * (double)i / (double)(M - 1);
        s->cnode[M - 1] = hi;
        s->M = M;
        s->mo = -1;
        for (int i = 0; i < M; ++i) if (s->cnode[i] == co) s->mo = i;
        return OR_OK;
    }
    if (co < lo || co > hi) return OR_E_LAYER;
    int sb;
    if (co == lo) sb = 0;
    else if (co == hi) sb = M - 1;
    else {
        if (M < 3) M = 3;
        double x = (co - lo) / (hi - lo) * (double)(M - 1);
        sb = (int)ceil(x - 0.5);                 /* round half down */
        if (sb < 1) sb = 1;
        if (sb > M - 2) sb = M - 2;
    }
    for (int i = 0; i < sb; ++i) s->cnode[i] = lo + (co - lo) * (double)i / (double)sb;
    s->cnode[sb] = co;
    for (int i = sb + 1; i < M; ++i)
        s->cnode[i] = co + (hi - co) * (double)(i - sb) / (double)(M - 1 - sb);
    s->cnode[M - 1] = (sb == M - 1) ? co : hi;
    s->M = M;
    s->mo = sb;
    return OR_OK;
}

/* Layer nodes zeta_0 = 0 < zeta_1 < ... < zeta_Mt = zeta_max, equidistant
 * unless given. */
static int layer_nodes(const or_problem* p, or_setup_t* s) {
    int Mt = p->m_layer;
    if (Mt < 1 || Mt > 64) return OR_E_INVALID;
    s->znode[0] = 0.0;
    if (p->nodes_zeta) {
        for (int j = 1; j <= Mt; ++j) {
            s->znode[j] = p->nodes_zeta[j - 1];
            if (!(s->znode[j] > s->znode[j - 1])) return OR_E_INVALID;
        }
    } else {
        for (int j = 1; j <= Mt; ++j) s->znode[j] = s->zmax * (double)j / (double)Mt;
        s->znode[Mt] = s->zmax;
    }
    s->Mt = Mt;
    return OR_OK;
}

/* Hat basis on increasing nodes t[0..m-1], evaluated at x clamped to the node
 * range: value of the m-th hat function. */
static double hat(const double* t, int m, int idx, double x) {
    if (m == 1) return 1.0;
    if (x < t[0]) x = t[0];
    if (x > t[m - 1]) x = t[m - 1];
    if (idx > 0 && x >= t[idx - 1] && x <= t[idx])
        return (x - t[idx - 1]) / (t[idx] - t[idx - 1]);
    if (idx < m - 1 && x >= t[idx] && x <= t[idx + 1])
        return (t[idx + 1] - x) / (t[idx + 1] - t[idx]);
    return 0.0;
}

/* Higher-degree piecewise Lagrange basis on nodes t[0..m-1] (the other
 * polynomial strategies the paper mentions in Sections 1 and 4.3): on the
 * segment [t_s, t_{s+1}] holding x (clamped, s in [0, m-2]) the interpolant is the
 * degree-p polynomial through the p+1 consecutive nodes starting at
 * clamp(s - (p-1)/2, 0, m-1-p); basis function idx is its Lagrange factor for
 * node idx (zero if idx is not among them).  Every such polynomial takes the node
 * values at its nodes, so the interpolant is continuous and reproduces the nodes. */
static double lagrange(const double* t, int m, int p, int idx, double x) {
    if (m == 1) return 1.0;
    if (p > m - 1) p = m - 1;
    if (p <= 1) return hat(t, m, idx, x);
    if (x < t[0]) x = t[0];
    if (x > t[m - 1]) x = t[m - 1];
    int sg = 0;
    while (sg < m - 2 && t[sg + 1] <= x) ++sg;
    int st = sg - (p - 1) / 2;
    if (st < 0) st = 0;
    if (st > m - 1 - p) st = m - 1 - p;
    if (idx < st || idx > st + p) return 0.0;
    double l = 1.0;
    for (int k = st; k <= st + p; ++k)
        if (k != idx) l *= (x - t[k]) / (t[idx] - t[k]);
    return l;
}

/* Weights of all K nodes at one point, following Eqn. 405 with bases phi_m
 * (real nodes, functions of Re gamma: piecewise linear, or Lagrange of degree
 * s->order) and piecewise linear varphi_j (layer nodes, functions of Im gamma on
 * the nodes -c_o zeta_j). */
void or_point_weights(const or_setup_t* s, double c0, double cval, double zval, double* w) {
    double re = cval, im = -cval * zval;
    if (s->Mt == 0) {
        for (int m = 0; m < s->M; ++m) w[m] = lagrange(s->cnode, s->M, s->order, m, re);
        return;
    }
    /* varphi_j live on Im gamma in [-c_o zeta_max, 0]; use increasing nodes. */
    int nz = s->Mt + 1;
    double tz[65];
    for (int j = 0; j < nz; ++j) tz[j] = -c0 * s->znode[nz - 1 - j];
    double phi0 = hat(tz, nz, nz - 1, im);
    for (int m = 0; m < s->M; ++m) w[m] = lagrange(s->cnode, s->M, s->order, m, re) * phi0;
    double phimo = lagrange(s->cnode, s->M, s->order, s->mo, re);
    for (int j = 1; j <= s->Mt; ++j) w[s->M + j - 1] = phimo * hat(tz, nz, nz - 1 - j, im);
}

/* Weights of the M x Ma real nodes at a point (no layer) in the bivariate
 * scheme: the tensor product of the hat functions of the speed nodes (in c) and
 * of the damping nodes (in a), the two-variable form of the interpolation of
 * Section 4.1 that the concluding remarks call for when a does not depend on c. */
void or_point_weights_ca(const or_setup_t* s, double cval, double aval, double* w) {
    for (int r = 0; r < s->Ma; ++r) {
        double ha = hat(s->anode, s->Ma, r, aval);
        for (int m = 0; m < s->M; ++m) w[m + s->M * r] = hat(s->cnode, s->M, m, cval) * ha;
    }
}

/* Weights of all K nodes at point i of the problem (any scheme).  The layer tensor
 * uses the same tensor-product hats with Im gamma = -c zeta on the second axis. */
static void point_weights_at(const or_problem* p, const or_setup_t* s, long i, double* w) {
    if (s->tensor) or_point_weights_ca(s, p->c[i], -p->c[i] * (p->zeta ? p->zeta[i] : 0.0), w);
    else if (s->Ma > 0) or_point_weights_ca(s, p->c[i], p->a ? p->a[i] : 0.0, w);
    else or_point_weights(s, p->c0, p->c[i], p->zeta ? p->zeta[i] : 0.0, w);
}

/* The floor a_floor on the symbol damping (reading of the standing assumption
 * a_min > 0 of Section 3, needed where a = 0): it applies to the nodes whose
 * speed is real, Im gamma_n = 0, whose symbol would otherwise vanish at
 * |xi| = omega / c_n.  Nodes with Im gamma_n < 0 (the absorbing layer) keep
 * their damping: their denominator has imaginary part 2 Re(gamma_n) |Im gamma_n|
 * |xi|^2 > 0 away from xi = 0.  P_N always keeps the true a. */
static void floor_real_nodes(const or_problem* p, or_setup_t* s) {
    for (int n = 0; n < s->K; ++n)
        if (s->gim[n] == 0.0 && s->ahat[n] < p->a_floor) s->ahat[n] = p->a_floor;
}

/* Set up nodes, per-node damping and per-node complex speed. */
int or_setup(const or_problem* p, or_setup_t* s) {
    memset(s, 0, sizeof(*s));
    if (p->interp_order < 0 || p->interp_order > 3) return OR_E_INVALID;
    s->order = p->interp_order < 1 ? 1 : p->interp_order;
    if (p->dim < 1 || p->dim > 3) return OR_E_SHAPE;
    /* even lengths (the frequency range -N/2..N/2-1 of reading A3) */
    for (int d = 0; d < p->dim; ++d) if (p->n[d] < 2 || p->n[d] % 2 || !(p->len[d] > 0)) return OR_E_SHAPE;
    long np = npoints(p);
    s->cmin = INFINITY; s->cmax = -INFINITY; s->zmax = 0.0;
    for (long i = 0; i < np; ++i) {
        double cv = p->c[i];
        if (!isfinite(cv) || !(cv > 0)) return OR_E_MEDIA;
        if (cv < s->cmin) s->cmin = cv;
        if (cv > s->cmax) s->cmax = cv;
        if (p->zeta) {
            double z = p->zeta[i];
            if (!isfinite(z) || z < 0) return OR_E_MEDIA;
            if (z > s->zmax) s->zmax = z;
        }
        if (p->a && (!isfinite(p->a[i]) || p->a[i] < 0)) return OR_E_MEDIA;
    }
    /* m_real = 1 asks for the one-node preconditioner Q_1 (Eqn. OneInterpPoint):
     * the single node c_o and no layer nodes. */
    int q1 = p->m_real == 1;
    int has_layer = s->zmax > 0.0 && !q1;
    /* Layer tensor: Re gamma = c on M equidistant nodes over [c_min, c_max] (c_o need
     * not be one), Im gamma = -c zeta on m_layer + 1 equidistant nodes over
     * [-max(c zeta), 0], node (m, r) with gamma = c_m + i g_r; the damping per speed
     * node as in the univariate scheme.  Piecewise linear, not with (c, a). */
    if (p->layer_tensor && has_layer) {
        if (p->m_damp >= 2 || s->order != 1 || p->m_layer < 1) return OR_E_INVALID;
        int rc = real_nodes(p, s, 0);
        if (rc) return rc;
        double gmax = 0.0;
        for (long i = 0; i < np; ++i) {
            double g = p->c[i] * (p->zeta ? p->zeta[i] : 0.0);
            if (g > gmax) gmax = g;
        }
        int Mi = p->m_layer + 1;
        for (int r = 0; r < Mi; ++r) s->anode[r] = -gmax + gmax * (double)r / (double)(Mi - 1);
        s->anode[Mi - 1] = 0.0;
        s->Ma = Mi;
        s->Mt = 0;
        s->tensor = 1;
        s->K = s->M * Mi;
        if (s->K > 64) return OR_E_INVALID;
        double a0 = p->a ? p->a[0] : 0.0, ahat[64];
        int uniform = 1;
        if (p->a) for (long i = 1; i < np; ++i) if (p->a[i] != a0) { uniform = 0; break; }
        for (int m = 0; m < s->M; ++m) ahat[m] = p->a_nodes ? p->a_nodes[m] : a0;
        if (!p->a_nodes && !uniform) {   /* hat(c)-weighted mean of a over the points */
            double num[64] = {0}, den[64] = {0}, mean = 0;
            for (long i = 0; i < np; ++i) {
                for (int m = 0; m < s->M; ++m) {
                    double h = hat(s->cnode, s->M, m, p->c[i]);
                    num[m] += h * p->a[i];
                    den[m] += h;
                }
                mean += p->a[i];
            }
            mean /= (double)np;
            for (int m = 0; m < s->M; ++m) ahat[m] = den[m] > 0 ? num[m] / den[m] : mean;
        }
        for (int r = 0; r < Mi; ++r)
            for (int m = 0; m < s->M; ++m) {
                int n = m + s->M * r;
                s->gre[n] = s->cnode[m];
                s->gim[n] = s->anode[r];
                s->ahat[n] = ahat[m];
            }
        floor_real_nodes(p, s);
        return OR_OK;
    }
    int rc = real_nodes(p, s, has_layer);
    if (rc) return rc;
    if (has_layer) {
        if (s->M + p->m_layer > 64) return OR_E_INVALID;
        rc = layer_nodes(p, s);
        if (rc) return rc;
    } else {
        s->Mt = 0;
    }
    s->K = s->M + s->Mt;
    if (s->K > 64) return OR_E_INVALID;

    /* Bivariate (c, a): damping nodes equidistant on [a_min, a_max] (a single
     * node when a is uniform), real node (m, r) = (c_m, a_r); no absorbing layer
     * (its nodes would need a third axis) and piecewise linear in both variables. */
    if (p->m_damp >= 2) {
        if (has_layer || s->order != 1 || p->m_damp > 64) return OR_E_INVALID;
        s->amin = INFINITY; s->amax = -INFINITY;
        for (long i = 0; i < np; ++i) {
            double av = p->a ? p->a[i] : 0.0;
            if (av < s->amin) s->amin = av;
            if (av > s->amax) s->amax = av;
        }
        int Ma = s->amax > s->amin ? p->m_damp : 1;
        for (int r = 0; r < Ma; ++r)
            s->anode[r] = Ma == 1 ? s->amin : s->amin + (s->amax - s->amin) * (double)r / (double)(Ma - 1);
        if (Ma > 1) s->anode[Ma - 1] = s->amax;
        s->Ma = Ma;
        s->K = s->M * Ma;
        if (s->K > 64) return OR_E_INVALID;
        for (int r = 0; r < Ma; ++r)
            for (int m = 0; m < s->M; ++m) {
                int n = m + s->M * r;
                s->gre[n] = s->cnode[m];
                s->gim[n] = 0.0;
                s->ahat[n] = s->anode[r];
            }
        floor_real_nodes(p, s);
        return OR_OK;
    }

    /* Symbol damping per real node: the symbol depends on x only through c,
     * so a must be a function of c (Section 4).  Uniform a is used as is;
     * given a(c_m) is used as given; otherwise the hat-weighted mean of a
     * over the points each real node serves.  Layer nodes take the damping
     * of c_o (before any floor). */
    int uniform = 1;
    double a0 = p->a ? p->a[0] : 0.0;
    if (p->a) for (long i = 1; i < np; ++i) if (p->a[i] != a0) { uniform = 0; break; }
    for (int m = 0; m < s->M; ++m) s->ahat[m] = a0;
    if (p->a_nodes) {
        for (int m = 0; m < s->M; ++m) s->ahat[m] = p->a_nodes[m];
    } else if (!uniform) {
        double num[64] = {0}, den[64] = {0}, w[128], mean = 0;
        for (long i = 0; i < np; ++i) {
            or_point_weights(s, p->c0, p->c[i], p->zeta ? p->zeta[i] : 0.0, w);
            for (int m = 0; m < s->M; ++m) { num[m] += w[m] * p->a[i]; den[m] += w[m]; }
            mean += p->a[i];
        }
        mean /= (double)np;
        for (int m = 0; m < s->M; ++m) s->ahat[m] = den[m] > 0 ? num[m] / den[m] : mean;
    }
    for (int m = 0; m < s->M; ++m) { s->gre[m] = s->cnode[m]; s->gim[m] = 0.0; }
    for (int j = 1; j <= s->Mt; ++j) {
        s->ahat[s->M + j - 1] = s->ahat[s->mo];
        s->gre[s->M + j - 1] = p->c0;                  /* gamma = c_o (1 - i zeta_j) */
        s->gim[s->M + j - 1] = -p->c0 * s->znode[j];
    }
    floor_real_nodes(p, s);
    /* Per-point check of the layer assumption: c = c_o where zeta > 0. */
    if (has_layer)
        for (long i = 0; i < np; ++i)
            if (p->zeta[i] > 0 && fabs(p->c[i] - p->c0) > 1e-12 * p->c0) return OR_E_LAYER;
    return OR_OK;
}

/* lambda(k) = |xi|^2 with xi_j = 2 pi k_j / L_j (Eqn. 021), or the stencil's own
 * symbol sum_j (4/h_j^2) sin^2(pi k_j / N_j).  k_j is the signed frequency of
 * DFT bin i_j: i_j for i_j < N_j/2, else i_j - N_j. */
static double lambda_of(const or_problem* p, const int* idx) {
    double lam = 0.0;
    for (int d = 0; d < p->dim; ++d) {
        int nn = p->n[d];
        int k = idx[d] < nn / 2 ? idx[d] : idx[d] - nn;
        if (p->symbol == 0) {
            double xi = 2.0 * M_PI * (double)k / p->len[d];
            lam += xi * xi;
        } else {
            double h = p->len[d] / (double)nn;
            double sn = sin(M_PI * (double)k / (double)nn);
            lam += 4.0 / (h * h) * sn * sn;
        }
    }
    return lam;
}

static void unravel(const or_problem* p, long i, int* idx) {
    for (int d = p->dim - 1; d >= 0; --d) { idx[d] = (int)(i % p->n[d]); i /= p->n[d]; }
}

/* Principal symbol q_{-2} = 1/(omega^2 + i omega a - gamma^2 lambda) (Eqn. 021). */
static cx symbol_q(double omega, double ahat, cx gamma, double lam) {
    cx den = omega * omega + I * omega * ahat - gamma * gamma * lam;
    return 1.0 / den;
}

/* u = Q_M v (Eqn. 403): one forward transform, then for every node n the
 * inverse transform of q_n * v^, added with the weight of node n at each x.
 * v, u: nrhs fields of N^d points. */
int or_apply(const or_problem* p, int nrhs, const cx* v, cx* u) {
    or_setup_t s;
    int rc = or_setup(p, &s);
    if (rc) return rc;
    long np = npoints(p);
    cx* vh = (cx*)malloc(sizeof(cx) * (size_t)np);
    cx* z = (cx*)malloc(sizeof(cx) * (size_t)np);
    double* lam = (double*)malloc(sizeof(double) * (size_t)np);
    double* wgt = (double*)malloc(sizeof(double) * (size_t)np * (size_t)s.K);
    if (!vh || !z || !lam || !wgt) { free(vh); free(z); free(lam); free(wgt); return OR_E_NOMEM; }
    int idx[3];
    for (long i = 0; i < np; ++i) { unravel(p, i, idx); lam[i] = lambda_of(p, idx); }
    for (long i = 0; i < np; ++i) point_weights_at(p, &s, i, wgt + i * s.K);
    for (int n = 0; n < s.K; ++n) {      /* zero denominators are rejected */
        cx g = s.gre[n] + I * s.gim[n];
        for (long i = 0; i < np; ++i) {
            cx den = p->omega * p->omega + I * p->omega * s.ahat[n] - g * g * lam[i];
            if (den == 0) { free(vh); free(z); free(lam); free(wgt); return OR_E_MEDIA; }
        }
    }
    for (int r = 0; r < nrhs; ++r) {
        const cx* vr = v + (long)r * np;
        cx* ur = u + (long)r * np;
        memcpy(vh, vr, sizeof(cx) * (size_t)np);
        or_fftnd(p->dim, p->n, vh, 0);
        for (long i = 0; i < np; ++i) ur[i] = 0;
        for (int n = 0; n < s.K; ++n) {
            cx g = s.gre[n] + I * s.gim[n];
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
            for (long i = 0; i < np; ++i) z[i] = symbol_q(p->omega, s.ahat[n], g, lam[i]) * vh[i];
            or_fftnd(p->dim, p->n, z, 1);
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
            for (long i = 0; i < np; ++i) ur[i] += wgt[i * s.K + n] * z[i];
        }
    }
    free(vh); free(z); free(lam); free(wgt);
    return OR_OK;
}

/* The exact operator Q of Eqn. Precond, discretised on the grid by brute force:
 * (Q v)(x) = N^-d sum_k q(gamma(x), a(x), xi_k) v^(k) exp(+i xi_k . x).
 * O(N^2d); only for small grids. */
int or_exact_psdo(const or_problem* p, const cx* v, cx* u) {
    long np = npoints(p);
    cx* vh = (cx*)malloc(sizeof(cx) * (size_t)np);
    if (!vh) return OR_E_NOMEM;
    memcpy(vh, v, sizeof(cx) * (size_t)np);
    or_fftnd(p->dim, p->n, vh, 0);
    int ix[3], ik[3];
    for (long i = 0; i < np; ++i) {
        unravel(p, i, ix);
        cx gam = p->c[i] * (1.0 - I * (p->zeta ? p->zeta[i] : 0.0));
        double ai = p->a ? p->a[i] : 0.0;
        if (cimag(gam) == 0.0 && ai < p->a_floor) ai = p->a_floor;   /* floored where the speed is real */
        cx acc = 0;
        for (long k = 0; k < np; ++k) {
            unravel(p, k, ik);
            double ph = 0.0;
            for (int d = 0; d < p->dim; ++d)
                ph += 2.0 * M_PI * (double)(((long)ix[d] * ik[d]) % p->n[d]) / (double)p->n[d];
            acc += symbol_q(p->omega, ai, gam, lambda_of(p, ik)) * vh[k] * (cos(ph) + I * sin(ph));
        }
        u[i] = acc / (double)np;
    }
    free(vh);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Finite-difference Helmholtz operator P_N (Section 5).               */
/* (P u)(x) = gamma^2 sum_j [u(x+h e_j) - 2u(x) + u(x-h e_j)]/h_j^2      */
/*          + (omega^2 + i omega a) u(x), indices periodic.            */
/* ------------------------------------------------------------------ */
int or_matvec(const or_problem* p, int nrhs, const cx* u, cx* y) {
    long np = npoints(p);
    long stride[3] = {1, 1, 1};
    for (int d = p->dim - 2; d >= 0; --d) stride[d] = stride[d + 1] * p->n[d + 1];
    for (int r = 0; r < nrhs; ++r) {
        const cx* ur = u + (long)r * np;
        cx* yr = y + (long)r * np;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (long i = 0; i < np; ++i) {
            int idx[3];
            unravel(p, i, idx);
            cx lap = 0;
            for (int d = 0; d < p->dim; ++d) {
                int nn = p->n[d];
                long ip = i + (long)(((idx[d] + 1) % nn) - idx[d]) * stride[d];
                long im = i + (long)(((idx[d] - 1 + nn) % nn) - idx[d]) * stride[d];
                double h = p->len[d] / (double)nn;
                lap += (ur[ip] - 2.0 * ur[i] + ur[im]) / (h * h);
            }
            cx gam = p->c[i] * (1.0 - I * (p->zeta ? p->zeta[i] : 0.0));
            double ai = p->a ? p->a[i] : 0.0;
            yr[i] = gam * gam * lap + (p->omega * p->omega + I * p->omega * ai) * ur[i];
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Restarted GMRES(m) (Saad and Schultz 1986), x0 given.               */
/* side = 0: right preconditioning   P Q y = f, x = Q y                */
/* side = 1: left preconditioning    Q P x = Q f  (Eqn. MainDiscretePrecond) */
/* side = 2: no preconditioner                                          */
/* Modified Gram-Schmidt Arnoldi, Givens rotations on the Hessenberg    */
/* matrix.  A cycle stops early when the rotated residual estimate      */
/* |g_{j+1}| drops below the target or on breakdown.  At each restart   */
/* the true residual ||f - P x|| / ||f|| is recomputed and decides      */
/* convergence.                                                          */
/* ------------------------------------------------------------------ */
static double nrm2(long n, const cx* x) {
    double s = 0;
#ifdef _OPENMP
#pragma omp parallel for reduction(+ : s) schedule(static)
#endif
    for (long i = 0; i < n; ++i) s += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
    return sqrt(s);
}
static cx dotc(long n, const cx* x, const cx* y) {     /* x^H y */
    double sr = 0, si = 0;
#ifdef _OPENMP
#pragma omp parallel for reduction(+ : sr, si) schedule(static)
#endif
    for (long i = 0; i < n; ++i) {
        cx t = conj(x[i]) * y[i];
        sr += creal(t);
        si += cimag(t);
    }
    return sr + I * si;
}

/* w -= h v over n points */
static void axpy_sub(long n, cx h, const cx* v, cx* w) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (long t = 0; t < n; ++t) w[t] -= h * v[t];
}

/* Threads the library uses (1 unless built with OpenMP). */
int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

typedef struct {
    int iters;          /* Arnoldi steps taken in total */
    int cycles;
    double rel_true_residual;
    int status;
    double rel_prec_residual;   /* residual of the system GMRES is applied to:
                                   ||Q(f - P x)|| / ||Q f|| for left, else the true one */
} or_solve_info;

/* Operator of the Krylov space: side 0: P Q, side 1: Q P, side 2: P. */
static int krylov_op(const or_problem* p, int side, const cx* v, cx* w, cx* tmp) {
    int rc;
    if (side == 0) { rc = or_apply(p, 1, v, tmp); if (rc) return rc; return or_matvec(p, 1, tmp, w); }
    if (side == 1) { rc = or_matvec(p, 1, v, tmp); if (rc) return rc; return or_apply(p, 1, tmp, w); }
    return or_matvec(p, 1, v, w);
}

/* One Arnoldi process of m steps from v0 (normalised inside); returns the
 * basis V (m+1 vectors) and the (m+1) x m Hessenberg H (row-major, ld m).
 * reorth = 1 repeats the Gram-Schmidt sweep once against the whole basis and
 * adds its coefficients to H (unconditional reorthogonalisation, as the
 * Arnoldi eigensolvers behind the condition numbers of Eqn. Cond use): the
 * basis then stays orthonormal to rounding after Ritz values have converged,
 * where one modified Gram-Schmidt sweep loses orthogonality.
 * Used directly by the invariant tests and the spectral diagnostics. */
int or_arnoldi(const or_problem* p, int side, int m, int reorth, const cx* v0, cx* V, cx* H, int* steps) {
    long np = npoints(p);
    cx* tmp = (cx*)malloc(sizeof(cx) * (size_t)np);
    if (!tmp) return OR_E_NOMEM;
    memset(H, 0, sizeof(cx) * (size_t)(m + 1) * (size_t)m);
    double b = nrm2(np, v0);
    for (long i = 0; i < np; ++i) V[i] = v0[i] / b;
    int j;
    for (j = 0; j < m; ++j) {
        cx* w = V + (long)(j + 1) * np;
        int rc = krylov_op(p, side, V + (long)j * np, w, tmp);
        if (rc) { free(tmp); return rc; }
        for (int i = 0; i <= j; ++i) {
            cx hij = dotc(np, V + (long)i * np, w);
            H[(long)i * m + j] = hij;
            axpy_sub(np, hij, V + (long)i * np, w);
        }
        if (reorth) {
            for (int i = 0; i <= j; ++i) {
                cx d = dotc(np, V + (long)i * np, w);
                H[(long)i * m + j] += d;
                axpy_sub(np, d, V + (long)i * np, w);
            }
        }
        double hn = nrm2(np, w);
        H[(long)(j + 1) * m + j] = hn;
        if (hn == 0.0) { j++; break; }
        for (long t = 0; t < np; ++t) w[t] /= hn;
    }
    *steps = j;
    free(tmp);
    return OR_OK;
}

int or_gmres(const or_problem* p, int side, int m, int max_cycles, double rtol,
             const cx* f, cx* x, or_solve_info* info, double* hist, int hist_len) {
    long np = npoints(p);
    memset(info, 0, sizeof(*info));
    if (m < 1 || m > 1000) return OR_E_INVALID;
    cx* V = (cx*)malloc(sizeof(cx) * (size_t)(m + 1) * (size_t)np);
    cx* r = (cx*)malloc(sizeof(cx) * (size_t)np);
    cx* tmp = (cx*)malloc(sizeof(cx) * (size_t)np);
    cx* H = (cx*)malloc(sizeof(cx) * (size_t)(m + 1) * (size_t)m);
    cx* g = (cx*)malloc(sizeof(cx) * (size_t)(m + 1));
    cx* cs = (cx*)malloc(sizeof(cx) * (size_t)m);
    cx* sn = (cx*)malloc(sizeof(cx) * (size_t)m);
    cx* y = (cx*)malloc(sizeof(cx) * (size_t)m);
    int rc = OR_OK;
    if (!V || !r || !tmp || !H || !g || !cs || !sn || !y) { rc = OR_E_NOMEM; goto done; }
    double fn = nrm2(np, f);
    if (fn == 0.0) { memset(x, 0, sizeof(cx) * (size_t)np); info->status = OR_OK; goto done; }
    double qfn = fn;
    if (side == 1) {
        rc = or_apply(p, 1, f, tmp); if (rc) goto done;
        qfn = nrm2(np, tmp);
    }
    int nh = 0;
    for (int cyc = 0; cyc < max_cycles; ++cyc) {
        /* true residual r = f - P x; with left preconditioning GMRES works on the
         * system Q P x = Q f (Eqn. MainDiscretePrecond), whose residual Q r decides */
        rc = or_matvec(p, 1, x, tmp); if (rc) goto done;
        for (long i = 0; i < np; ++i) r[i] = f[i] - tmp[i];
        double rel = nrm2(np, r) / fn;
        info->rel_true_residual = rel;
        if (side == 1) { rc = or_apply(p, 1, r, tmp); if (rc) goto done; memcpy(r, tmp, sizeof(cx) * (size_t)np); }
        double beta = nrm2(np, r);
        double trel = side == 1 ? beta / qfn : rel;
        info->rel_prec_residual = trel;
        if (hist && nh < hist_len) hist[nh++] = trel;
        if (trel <= rtol) { info->status = OR_OK; goto done; }
        info->cycles++;
        double target = rtol * (side == 1 ? qfn : fn);
        for (long i = 0; i < np; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0;
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            cx* w = V + (long)(j + 1) * np;
            rc = krylov_op(p, side, V + (long)j * np, w, tmp); if (rc) goto done;
            double w0 = nrm2(np, w);
            for (int i = 0; i <= j; ++i) {                      /* modified Gram-Schmidt */
                cx hij = dotc(np, V + (long)i * np, w);
                H[(long)i * m + j] = hij;
                axpy_sub(np, hij, V + (long)i * np, w);
            }
            double hn = nrm2(np, w);
            H[(long)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {                       /* previous rotations */
                cx a = H[(long)i * m + j], b = H[(long)(i + 1) * m + j];
                H[(long)i * m + j] = conj(cs[i]) * a + conj(sn[i]) * b;
                H[(long)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            {                                                    /* new rotation */
                cx a = H[(long)j * m + j];
                double bb = hn;
                double den = sqrt(creal(a) * creal(a) + cimag(a) * cimag(a) + bb * bb);
                cx c_, s_;
                if (den == 0.0) { c_ = 1; s_ = 0; }
                else if (cabs(a) == 0.0) { c_ = 0; s_ = 1; }
                else { c_ = a / den; s_ = bb / den; }
                cs[j] = c_; sn[j] = s_;
                H[(long)j * m + j] = conj(c_) * a + conj(s_) * bb;
                H[(long)(j + 1) * m + j] = 0;
                cx gj = g[j];
                g[j] = conj(c_) * gj;
                g[j + 1] = -s_ * gj;
            }
            k = j + 1;
            info->iters++;
            if (cabs(g[j + 1]) <= target || hn <= 1e-14 * w0) break;
            for (long t = 0; t < np; ++t) w[t] /= hn;
        }
        for (int i = k - 1; i >= 0; --i) {                      /* back substitution */
            cx s = g[i];
            for (int l = i + 1; l < k; ++l) s -= H[(long)i * m + l] * y[l];
            y[i] = s / H[(long)i * m + i];
        }
        for (long t = 0; t < np; ++t) {
            cx s = 0;
            for (int i = 0; i < k; ++i) s += y[i] * V[(long)i * np + t];
            r[t] = s;
        }
        if (side == 0) { rc = or_apply(p, 1, r, tmp); if (rc) goto done; for (long t = 0; t < np; ++t) x[t] += tmp[t]; }
        else for (long t = 0; t < np; ++t) x[t] += r[t];
    }
    rc = or_matvec(p, 1, x, tmp); if (rc) goto done;
    for (long i = 0; i < np; ++i) r[i] = f[i] - tmp[i];
    info->rel_true_residual = nrm2(np, r) / fn;
    info->rel_prec_residual = info->rel_true_residual;
    if (side == 1) {
        rc = or_apply(p, 1, r, tmp); if (rc) goto done;
        info->rel_prec_residual = nrm2(np, tmp) / qfn;
    }
    if (hist && nh < hist_len) hist[nh++] = info->rel_prec_residual;
    info->status = info->rel_prec_residual <= rtol ? OR_OK : OR_E_NOT_CONVERGED;
    rc = info->status;
done:
    free(V); free(r); free(tmp); free(H); free(g); free(cs); free(sn); free(y);
    return rc;
}

/* Size of or_setup_t for the Python side to check its mirror of the struct. */
int or_setup_sizeof(void) { return (int)sizeof(or_setup_t); }
int or_problem_sizeof(void) { return (int)sizeof(or_problem); }
