// Host side of the spectral diagnostics: eigenvalues of the small Hessenberg
// matrix an Arnoldi process returns (Ritz values, which approach the
// eigenvalues of largest modulus first, and harmonic Ritz values, which
// approach those nearest zero first), the two ends of the spectral condition
// number of Eqn. Cond (Section 5).  Dense work on at most 64 x 64 matrices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>
#include <vector>

#include "../../include/helmpre.h"

namespace {

using C = std::complex<double>;

// Eigenvalues of the n x n upper Hessenberg matrix a (row-major, overwritten)
// by the shifted QR algorithm: Givens-rotation QR steps with the Wilkinson
// shift of the trailing 2 x 2 block, deflation at negligible subdiagonal
// entries, an exceptional shift after ten steps without one.  Returns false if
// an eigenvalue has not deflated after 60 steps.
bool hessenberg_eigenvalues(std::vector<C>& a, int n, C* w) {
  const double eps = std::numeric_limits<double>::epsilon();
  auto A = [&](int i, int j) -> C& { return a[(size_t)i * n + j]; };
  double anorm = 0.0;
  for (const C& z : a) anorm = std::max(anorm, std::abs(z));
  std::vector<C> cs(n), sn(n);
  int hi = n - 1, since = 0;
  while (hi >= 0) {
    int lo = hi;
    while (lo > 0) {
      double s = std::abs(A(lo, lo)) + std::abs(A(lo - 1, lo - 1));
      if (s == 0.0) s = anorm;
      if (std::abs(A(lo, lo - 1)) <= eps * s) {
        A(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {   // a 1 x 1 block has deflated
      w[hi] = A(hi, hi);
      --hi;
      since = 0;
      continue;
    }
    if (++since > 60) return false;
    C mu;
    if (since % 11 == 10) {
      mu = A(hi, hi) + std::abs(A(hi, hi - 1)) + (hi - 1 > lo ? std::abs(A(hi - 1, hi - 2)) : 0.0);
    } else {
      const C p = A(hi - 1, hi - 1), q = A(hi - 1, hi), r = A(hi, hi - 1), t = A(hi, hi);
      const C half = 0.5 * (p + t);
      const C disc = std::sqrt(0.25 * (p - t) * (p - t) + q * r);
      const C e1 = half + disc, e2 = half - disc;
      mu = std::abs(e1 - t) <= std::abs(e2 - t) ? e1 : e2;
    }
    for (int i = lo; i <= hi; ++i) A(i, i) -= mu;
    // A - mu I = G^H R: rotation k zeroes the subdiagonal entry of column k
    for (int k = lo; k < hi; ++k) {
      const C x = A(k, k), y = A(k + 1, k);
      const double r = std::hypot(std::abs(x), std::abs(y));
      const C c = r == 0.0 ? C(1.0) : x / r, s = r == 0.0 ? C(0.0) : y / r;
      cs[k] = c;
      sn[k] = s;
      for (int j = k; j <= hi; ++j) {
        const C u = A(k, j), v = A(k + 1, j);
        A(k, j) = std::conj(c) * u + std::conj(s) * v;
        A(k + 1, j) = -s * u + c * v;
      }
    }
    // R G^H + mu I
    for (int k = lo; k < hi; ++k) {
      const C c = cs[k], s = sn[k];
      for (int i = lo; i <= k + 1; ++i) {
        const C u = A(i, k), v = A(i, k + 1);
        A(i, k) = u * c + v * s;
        A(i, k + 1) = -u * std::conj(s) + v * std::conj(c);
      }
    }
    for (int i = lo; i <= hi; ++i) A(i, i) += mu;
  }
  return true;
}

// Solve M^H f = e_{n-1} for the n x n matrix m (row-major) by Gaussian
// elimination with partial pivoting; false if M is singular.
bool solve_adjoint_last(const std::vector<C>& m, int n, std::vector<C>& f) {
  std::vector<C> b((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) b[(size_t)i * n + j] = std::conj(m[(size_t)j * n + i]);
  f.assign(n, 0.0);
  f[n - 1] = 1.0;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(b[(size_t)i * n + k]) > std::abs(b[(size_t)piv * n + k])) piv = i;
    if (b[(size_t)piv * n + k] == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(b[(size_t)k * n + j], b[(size_t)piv * n + j]);
      std::swap(f[k], f[piv]);
    }
    for (int i = k + 1; i < n; ++i) {
      const C l = b[(size_t)i * n + k] / b[(size_t)k * n + k];
      if (l == 0.0) continue;
      for (int j = k; j < n; ++j) b[(size_t)i * n + j] -= l * b[(size_t)k * n + j];
      f[i] -= l * f[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    C s = f[i];
    for (int j = i + 1; j < n; ++j) s -= b[(size_t)i * n + j] * f[j];
    f[i] = s / b[(size_t)i * n + i];
  }
  return true;
}

// Solve (A - mu I) x = b in place for the n x n upper Hessenberg matrix a
// (row-major) by Gaussian elimination with partial pivoting between adjacent rows
// (the only rows a column's elimination touches); a zero pivot is replaced by
// tiny, which makes the solve an inverse-iteration step at an exact eigenvalue.
void hessenberg_shifted_solve(const std::vector<C>& a, int n, C mu, double tiny, std::vector<C>& x) {
  std::vector<C> b(a);
  for (int i = 0; i < n; ++i) b[(size_t)i * n + i] -= mu;
  for (int c = 0; c + 1 < n; ++c) {
    C* r0 = &b[(size_t)c * n];
    C* r1 = &b[(size_t)(c + 1) * n];
    if (std::abs(r1[c]) > std::abs(r0[c])) {
      for (int j = c; j < n; ++j) std::swap(r0[j], r1[j]);
      std::swap(x[c], x[c + 1]);
    }
    if (r0[c] == 0.0) r0[c] = tiny;
    const C l = r1[c] / r0[c];
    if (l != 0.0) {
      for (int j = c; j < n; ++j) r1[j] -= l * r0[j];
      x[c + 1] -= l * x[c];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    C sacc = x[i];
    for (int j = i + 1; j < n; ++j) sacc -= b[(size_t)i * n + j] * x[j];
    C d = b[(size_t)i * n + i];
    if (d == 0.0) d = tiny;
    x[i] = sacc / d;
  }
}

double norm2(const std::vector<C>& x) {
  double s = 0.0;
  for (const C& z : x) s += std::norm(z);
  return std::sqrt(s);
}

}  // namespace

extern "C" hp_status hp_ritz_values(const void* H, int m, int k, int harmonic, void* theta, void* Y,
                                    double* resid) {
  if (!H || !theta || m < 1 || m > 64 || k < 1 || k > m || (harmonic != 0 && harmonic != 1)) return HP_E_INVALID;
  const C* h = (const C*)H;
  std::vector<C> a((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      const C v = h[(size_t)i * m + j];
      if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return HP_E_NONFINITE;
      a[(size_t)i * k + j] = j + 1 >= i ? v : C(0.0);
    }
  if (harmonic) {
    // H_k + |h_{k+1,k}|^2 f e_k^T with H_k^H f = e_k: only the last column changes,
    // the matrix stays upper Hessenberg
    const double beta = std::abs(h[(size_t)k * m + (k - 1)]);
    std::vector<C> f;
    if (!solve_adjoint_last(a, k, f)) return HP_E_INVALID;
    for (int i = 0; i < k; ++i) a[(size_t)i * k + (k - 1)] += beta * beta * f[i];
  }
  std::vector<C> work(a);
  C* th = (C*)theta;
  if (!hessenberg_eigenvalues(work, k, th)) return HP_E_NOT_CONVERGED;
  if (!Y && !resid) return HP_OK;
  // vectors by two steps of inverse iteration, residuals in the Arnoldi relation:
  // || A V_k y - theta V_k y || = || Hbar_k y - theta [y; 0] || for orthonormal V
  double anorm = 0.0;
  for (const C& z : a) anorm = std::max(anorm, std::abs(z));
  const double tiny = std::max(anorm, 1e-300) * std::numeric_limits<double>::epsilon();
  std::vector<C> y(k);
  for (int i = 0; i < k; ++i) {
    for (int r = 0; r < k; ++r) y[r] = C(1.0, 0.0) / std::sqrt((double)k);
    for (int it = 0; it < 2; ++it) {
      hessenberg_shifted_solve(a, k, th[i], tiny, y);
      const double nr = norm2(y);
      if (!(nr > 0.0) || !std::isfinite(nr)) return HP_E_NOT_CONVERGED;
      for (C& z : y) z /= nr;
    }
    if (Y)
      for (int r = 0; r < k; ++r) ((C*)Y)[(size_t)i * k + r] = y[r];
    if (resid) {
      double s2 = 0.0;
      for (int r = 0; r <= k; ++r) {
        C acc = r < k ? -th[i] * y[r] : C(0.0);
        for (int c = std::max(0, r - 1); c < k; ++c) acc += h[(size_t)r * m + c] * y[c];
        s2 += std::norm(acc);
      }
      resid[i] = std::sqrt(s2);
    }
  }
  return HP_OK;
}

// Explicitly restarted Arnoldi for one end of the spectrum (Section 5, Eqn. Cond).
// The largest modulus: Ritz values of the operator itself.  The smallest: the largest
// Ritz value of the inverse operator (shift-invert at zero), whose applications are
// inner GMRES solves; P_N Q and Q P_N are similar (Q is invertible), so both use
// (Q P_N)^{-1}.  Each run of m steps restarts from the wanted Ritz vector V_k y until
// its residual relative to |theta| is <= tol.
extern "C" hp_status hp_extreme_eigenvalue(hp_plan p, const void* v0, int m, int side, int smallest,
                                           int max_restarts, double tol, void* lambda, double* rel_resid,
                                           int* runs, void* stream) {
  if (!p || !v0 || !lambda || !rel_resid || !runs || m < 2 || m > 64 || max_restarts < 0 ||
      (smallest != 0 && smallest != 1) || side < HP_RIGHT || side > HP_NONE || !(tol >= 0.0))
    return HP_E_INVALID;
  hp_plan_info info;
  hp_status rc = hp_plan_query(p, &info);
  if (rc != HP_OK) return rc;
  size_t npts = 1;
  for (int d = 0; d < info.dim; ++d) npts *= (size_t)info.n[d];
  const int op = smallest ? (side == HP_NONE ? HP_NONE_INVERSE : HP_LEFT_INVERSE) : side;
  void* start = nullptr;
  if (hipMalloc(&start, npts * sizeof(C)) != hipSuccess) return HP_E_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  rc = hipMemcpyAsync(start, v0, npts * sizeof(C), hipMemcpyDeviceToDevice, st) == hipSuccess ? HP_OK : HP_E_DEVICE;
  std::vector<C> H((size_t)(m + 1) * m), th(m), Y((size_t)m * m);
  std::vector<double> res(m);
  C best(0.0);
  double best_rel = INFINITY;
  bool inner_short = false;
  int r = 0;
  for (; rc == HP_OK && r <= max_restarts; ++r) {
    int k = 0;
    const hp_status arc = hp_arnoldi(p, start, m, op, H.data(), &k, stream);
    if (arc == HP_E_NOT_CONVERGED) inner_short = true;
    else if (arc != HP_OK) { rc = arc; break; }
    if (k == 0) { rc = HP_E_INVALID; break; }   // a zero start vector
    if ((rc = hp_ritz_values(H.data(), m, k, 0, th.data(), Y.data(), res.data())) != HP_OK) break;
    int w = 0;
    for (int i = 1; i < k; ++i)
      if (std::abs(th[i]) > std::abs(th[w])) w = i;
    best = th[w];
    best_rel = std::abs(th[w]) > 0.0 ? res[w] / std::abs(th[w]) : INFINITY;
    if (best_rel <= tol || k < m || r == max_restarts) { ++r; break; }
    rc = hp_arnoldi_vector(p, &Y[(size_t)w * k], k, start, stream);
  }
  (void)hipFree(start);
  if (rc != HP_OK) return rc;
  *(C*)lambda = smallest ? (std::abs(best) > 0.0 ? C(1.0) / best : C(INFINITY)) : best;
  *rel_resid = best_rel;
  *runs = r;
  return best_rel <= tol && !inner_short ? HP_OK : HP_E_NOT_CONVERGED;
}
