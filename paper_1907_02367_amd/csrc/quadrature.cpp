// Quadrature on the reference n-simplex.
//
// The method integrates only over n-simplices: spatial elements mapped to a
// tent's bottom and top facets and the vertical time-like faces (Sec. 2.4
// closing remark, Sec. 4.1 and its Fig. 2).  One rule on the reference
// simplex is built once and mapped everywhere.
//
// Rule: collapsed-coordinate (conical product) Gauss rule with q points per
// direction, exact for total degree <= 2q - 1:
//   xi_n = s_n with weight (1 - s_n)^(n-1), ..., xi_1 = s_1 (1-s_2)...(1-s_n).
// Point order: s_n slowest, s_1 fastest; 1D nodes ascending.
//
// 1D Gauss-Jacobi rules on [0,1] (weight (1-s)^a): the nodes are the
// eigenvalues of the symmetric tridiagonal Jacobi matrix of the monic Jacobi
// recurrence (Golub-Welsch), found here by Sturm-sequence bisection; each
// weight is the Christoffel number 1 / sum_k phat_k(x)^2 with phat_k the
// orthonormal polynomials, which equals mu_0 times the squared first
// component of the normalised eigenvector.
#include <cmath>

#include "tdg_internal.h"

namespace tdg {

namespace {

// number of eigenvalues of the tridiagonal (diag d, off-diagonal squared b2) below x
int sturm_count(const std::vector<double>& d, const std::vector<double>& b2, double x) {
  int cnt = 0;
  double q = d[0] - x;
  if (q < 0) cnt++;
  for (size_t i = 1; i < d.size(); ++i) {
    double qq = (q == 0.0) ? 1e-300 : q;
    q = (d[i] - x) - b2[i - 1] / qq;
    if (q < 0) cnt++;
  }
  return cnt;
}

}  // namespace

void gauss_jacobi01(int q, int a, std::vector<double>& x, std::vector<double>& w) {
  const double b = 0.0;
  std::vector<double> alpha(q), beta(q > 1 ? q - 1 : 0);
  for (int i = 0; i < q; ++i) {
    double s = 2.0 * i + a + b;
    alpha[i] = (i == 0) ? (b - a) / (a + b + 2.0) : (b * b - (double)a * a) / (s * (s + 2.0));
  }
  for (int i = 1; i < q; ++i) {
    double s = 2.0 * i + a + b;
    beta[i - 1] = 4.0 * i * (i + a) * (i + b) * (i + a + b) / (s * s * (s + 1.0) * (s - 1.0));
  }
  const double mu0 = std::pow(2.0, a + b + 1.0) * std::tgamma(a + 1.0) * std::tgamma(b + 1.0) / std::tgamma(a + b + 2.0);
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    // the i-th smallest eigenvalue lies in (-1, 1)
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
      double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (sturm_count(alpha, beta, mid) > i)
        hi = mid;
      else
        lo = mid;
    }
    double xi = 0.5 * (lo + hi);
    // Christoffel number from the orthonormal recurrence
    double p_prev = 0.0, p = 1.0 / std::sqrt(mu0), sum = p * p;
    for (int k = 0; k + 1 < q; ++k) {
      double sb = std::sqrt(beta[k]);
      double sb_prev = (k == 0) ? 0.0 : std::sqrt(beta[k - 1]);
      double pn = ((xi - alpha[k]) * p - sb_prev * p_prev) / sb;
      p_prev = p;
      p = pn;
      sum += p * p;
    }
    x[i] = 0.5 * (xi + 1.0);
    w[i] = (1.0 / sum) * std::pow(2.0, -a - 1.0);
  }
}

Quadrature simplex_rule(int n, int q) {
  Quadrature R;
  R.n = n;
  R.q = q;
  std::vector<std::vector<double>> xs(n + 1), ws(n + 1);
  for (int d = 1; d <= n; ++d) gauss_jacobi01(q, d - 1, xs[d], ws[d]);
  int Q = 1;
  for (int d = 0; d < n; ++d) Q *= q;
  R.Q = Q;
  R.lam.assign((size_t)Q * (n + 1), 0.0);
  R.w.assign(Q, 0.0);
  for (int idx = 0; idx < Q; ++idx) {
    // digit for s_n is the most significant
    int rem = idx;
    int digit[4] = {0, 0, 0, 0};
    for (int pos = n - 1; pos >= 0; --pos) {
      digit[pos] = rem % q;
      rem /= q;
    }
    double xi[4] = {0, 0, 0, 0};
    double wt = 1.0, scale = 1.0;
    for (int pos = 0; pos < n; ++pos) {
      int d = n - pos;  // pos 0 is s_n
      double s = xs[d][digit[pos]];
      wt *= ws[d][digit[pos]];
      xi[d - 1] = s * scale;
      scale *= (1.0 - s);
    }
    double sum = 0.0;
    for (int d = 0; d < n; ++d) sum += xi[d];
    R.lam[(size_t)idx * (n + 1)] = 1.0 - sum;
    for (int d = 0; d < n; ++d) R.lam[(size_t)idx * (n + 1) + 1 + d] = xi[d];
    R.w[idx] = wt;
  }
  return R;
}

}  // namespace tdg
