// Host FP64 dense linear algebra for the L x L projected problems of
// Rayleigh-Ritz (L <= a few hundred): Cholesky, triangular inverse, symmetric
// eigen-decomposition (Householder tridiagonalisation followed by implicit QL
// iterations with Wilkinson shifts), and the symmetric-definite generalised
// problem built from them.  All matrices are row-major with leading dimension n.
#include "dense_host.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace slrf {

bool chol_upper(int n, double* G) {
  // G = R^T R, R upper triangular, stored in the upper triangle of G; the
  // strict lower triangle is zeroed.
  for (int j = 0; j < n; ++j) {
    double d = G[j * n + j];
    for (int k = 0; k < j; ++k) d -= G[k * n + j] * G[k * n + j];
    if (!(d > 0.0)) return false;
    const double r = std::sqrt(d);
    G[j * n + j] = r;
    for (int i = j + 1; i < n; ++i) {
      double s = G[j * n + i];
      for (int k = 0; k < j; ++k) s -= G[k * n + j] * G[k * n + i];
      G[j * n + i] = s / r;
    }
    for (int i = 0; i < j; ++i) G[j * n + i] = 0.0;
  }
  return true;
}

void tri_upper_inverse(int n, double* R) {
  // In-place inverse of an upper-triangular matrix (column by column).
  for (int j = n - 1; j >= 0; --j) {
    const double rjj = 1.0 / R[j * n + j];
    R[j * n + j] = rjj;
    // column j of the inverse, rows i < j: x_i = -(sum_{k=i+1..j} R_ik x_k) / R_ii
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += R[i * n + k] * (k == j ? rjj : R[k * n + j]);
      R[i * n + j] = -s / R[i * n + i];
    }
  }
}

// Householder reduction of symmetric A (row-major) to tridiagonal form
// T = Q^T A Q with diagonal d and off-diagonal e (e[i] couples i and i+1).
// Q is returned in Z (row-major, Z[row * n + col]).
static void tridiagonalize(int n, std::vector<double>& A, std::vector<double>& d,
                           std::vector<double>& e, std::vector<double>& Z) {
  Z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  d.assign(n, 0.0);
  e.assign(n, 0.0);
  std::vector<double> v(n), p(n), q(n);
  for (int k = 0; k + 2 < n; ++k) {
    // reflect x = A[k+1:, k] onto a multiple of e_1
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += A[(size_t)i * n + k] * A[(size_t)i * n + k];
    alpha = std::sqrt(alpha);
    const double x0 = A[(size_t)(k + 1) * n + k];
    if (alpha == 0.0) continue;
    const double beta = x0 >= 0.0 ? -alpha : alpha;  // new subdiagonal value
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    v[k + 1] = x0 - beta;
    for (int i = k + 2; i < n; ++i) v[i] = A[(size_t)i * n + k];
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double tau = 2.0 / vv;
    // p = tau * A v on the trailing block (rows/cols k..n-1 affected)
    for (int i = k; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += A[(size_t)i * n + j] * v[j];
      p[i] = tau * s;
    }
    for (int i = 0; i < k; ++i) p[i] = 0.0;
    double pv = 0.0;
    for (int i = k + 1; i < n; ++i) pv += p[i] * v[i];
    const double K = 0.5 * tau * pv;
    for (int i = k; i < n; ++i) q[i] = p[i] - K * v[i];
    // A <- A - v q^T - q v^T on rows/cols >= k
    for (int i = k; i < n; ++i)
      for (int j = k; j < n; ++j)
        A[(size_t)i * n + j] -= v[i] * q[j] + q[i] * v[j];
    // accumulate Z <- Z H, H = I - tau v v^T
    for (int r = 0; r < n; ++r) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += Z[(size_t)r * n + j] * v[j];
      s *= tau;
      for (int j = k + 1; j < n; ++j) Z[(size_t)r * n + j] -= s * v[j];
    }
  }
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];
  e[n - 1] = 0.0;
}

// Implicit QL with Wilkinson shifts on (d, e), the published algorithm of the
// EISPACK routine tql2 (Bowdler, Martin, Reinsch and Wilkinson, 1968); rotations
// accumulated in Z.
static bool tridiag_ql(int n, std::vector<double>& d, std::vector<double>& e,
                       std::vector<double>& Z) {
  const double eps = 2.220446049250313e-16;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    for (;;) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (++iter > 60) return false;
      // Wilkinson-type shift from the leading 2x2 block
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        const double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {
          const double zf = Z[(size_t)k * n + i + 1];
          const double zi = Z[(size_t)k * n + i];
          Z[(size_t)k * n + i + 1] = s * zi + c * zf;
          Z[(size_t)k * n + i] = c * zi - s * zf;
        }
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

bool sym_eig(int n, const double* A, double* w, double* V) {
  if (n == 0) return true;
  std::vector<double> a(A, A + (size_t)n * n), d, e, Z;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      const double s = 0.5 * (a[(size_t)i * n + j] + a[(size_t)j * n + i]);
      a[(size_t)i * n + j] = a[(size_t)j * n + i] = s;
    }
  tridiagonalize(n, a, d, e, Z);
  if (!tridiag_ql(n, d, e, Z)) return false;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return d[x] < d[y]; });
  for (int j = 0; j < n; ++j) {
    w[j] = d[order[j]];
    for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = Z[(size_t)i * n + order[j]];
  }
  return true;
}

int sym_gen_eig(int n, const double* Ah, const double* Bh, double* theta, double* S,
                int* used_fallback) {
  // (Ah) s = theta (Bh) s, S^T Bh S = I, theta ascending.  Returns the number
  // of Ritz pairs (n normally; fewer if Bh had to be truncated), or -1.
  if (used_fallback) *used_fallback = 0;
  if (n == 0) return 0;
  std::vector<double> R(Bh, Bh + (size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      const double s = 0.5 * (R[(size_t)i * n + j] + R[(size_t)j * n + i]);
      R[(size_t)i * n + j] = R[(size_t)j * n + i] = s;
    }
  std::vector<double> T;  // n x k transformation with T^T Bh T = I
  int k = n;
  std::vector<double> Rc = R;
  if (chol_upper(n, Rc.data())) {
    tri_upper_inverse(n, Rc.data());  // R^{-1}, upper
    T = Rc;
  } else {
    // Fallback: Bh = W diag(mu) W^T, keep mu > 1e-14 max(mu), T = W mu^{-1/2}
    if (used_fallback) *used_fallback = 1;
    std::vector<double> mu(n), W((size_t)n * n);
    if (!sym_eig(n, R.data(), mu.data(), W.data())) return -1;
    const double mmax = mu[n - 1];
    if (!(mmax > 0.0)) return -1;
    std::vector<int> keep;
    for (int i = 0; i < n; ++i)
      if (mu[i] > 1e-14 * mmax) keep.push_back(i);
    k = (int)keep.size();
    T.assign((size_t)n * k, 0.0);
    for (int c = 0; c < k; ++c) {
      const double sc = 1.0 / std::sqrt(mu[keep[c]]);
      for (int i = 0; i < n; ++i) T[(size_t)i * k + c] = W[(size_t)i * n + keep[c]] * sc;
    }
  }
  // Cm = T^T Ah T (k x k)
  std::vector<double> AT((size_t)n * k, 0.0), Cm((size_t)k * k, 0.0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < n; ++l) {
      const double a = Ah[(size_t)i * n + l];
      if (a == 0.0) continue;
      for (int c = 0; c < k; ++c) AT[(size_t)i * k + c] += a * T[(size_t)l * k + c];
    }
  for (int r = 0; r < k; ++r)
    for (int i = 0; i < n; ++i) {
      const double t = T[(size_t)i * k + r];
      if (t == 0.0) continue;
      for (int c = 0; c < k; ++c) Cm[(size_t)r * k + c] += t * AT[(size_t)i * k + c];
    }
  std::vector<double> w(k), Wv((size_t)k * k);
  if (!sym_eig(k, Cm.data(), w.data(), Wv.data())) return -1;
  // S = T Wv (n x k) written into n x n S (columns >= k zero)
  for (size_t i = 0; i < (size_t)n * n; ++i) S[i] = 0.0;
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < k; ++l) {
      const double t = T[(size_t)i * k + l];
      if (t == 0.0) continue;
      for (int c = 0; c < k; ++c) S[(size_t)i * n + c] += t * Wv[(size_t)l * k + c];
    }
  for (int c = 0; c < k; ++c) theta[c] = w[c];
  for (int c = k; c < n; ++c) theta[c] = HUGE_VAL;
  return k;
}

}  // namespace slrf
