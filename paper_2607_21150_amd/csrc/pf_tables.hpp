// One-dimensional reference tables for tensor-product hexahedra (host side).
//
// Nodes are Gauss-Lobatto-Legendre points (end points plus the roots of P_p'),
// quadrature points are Gauss-Legendre points; both are found by Newton's
// method on the Legendre recurrence from Chebyshev-type initial guesses. The
// Lagrange basis is evaluated in barycentric form and its derivative through
// the nodal differentiation matrix (exact, since the derivative has degree p-1).
#pragma once
#include <cmath>
#include <vector>

namespace pfmf {

struct Legendre {
  // P_n and P_n' at x via the three-term recurrence.
  static void eval(int n, long double x, long double& p, long double& dp) {
    long double pm = 1.0L, pc = x;
    if (n == 0) { p = 1.0L; dp = 0.0L; return; }
    for (int k = 1; k < n; ++k) {
      long double pn = ((2 * k + 1) * x * pc - k * pm) / (k + 1);
      pm = pc;
      pc = pn;
    }
    p = pc;
    // (1 - x^2) P_n' = n (P_{n-1} - x P_n)
    dp = n * (pm - x * pc) / (1.0L - x * x);
  }
};

inline void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double t = -std::cos(pi * (i + 0.75L) / (n + 0.5L));
    for (int it = 0; it < 100; ++it) {
      long double p, dp;
      Legendre::eval(n, t, p, dp);
      long double dt = p / dp;
      t -= dt;
      if (std::fabs((double)dt) < 1e-19) break;
    }
    long double p, dp;
    Legendre::eval(n, t, p, dp);
    x[i] = (double)t;
    w[i] = (double)(2.0L / ((1.0L - t * t) * dp * dp));
  }
}

// GLL points: -1, roots of P_{n-1}', +1 (Newton on P_{n-1}' with P_{n-1}'' from
// the Legendre ODE (1-x^2) y'' = 2 x y' - m (m+1) y).
inline void gauss_lobatto(int n, std::vector<double>& x) {
  x.assign(n, 0.0);
  x[0] = -1.0;
  x[n - 1] = 1.0;
  const int m = n - 1;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 1; i < n - 1; ++i) {
    long double t = -std::cos(pi * i / m);
    for (int it = 0; it < 100; ++it) {
      long double p, dp;
      Legendre::eval(m, t, p, dp);
      long double d2p = (2.0L * t * dp - m * (m + 1.0L) * p) / (1.0L - t * t);
      long double dt = dp / d2p;
      t -= dt;
      if (std::fabs((double)dt) < 1e-19) break;
    }
    x[i] = (double)t;
  }
}

// B[q][i] = l_i(xq_q), D[q][i] = l_i'(xq_q) for Lagrange polynomials on nodes xn.
inline void lagrange_tables(const std::vector<double>& xn, const std::vector<double>& xq,
                            std::vector<double>& B, std::vector<double>& D) {
  const int P = (int)xn.size(), Q = (int)xq.size();
  std::vector<long double> bw(P, 1.0L);  // barycentric weights
  for (int j = 0; j < P; ++j)
    for (int k = 0; k < P; ++k)
      if (k != j) bw[j] /= ((long double)xn[j] - xn[k]);
  // nodal differentiation matrix Dn[j][i] = l_i'(x_j)
  std::vector<long double> Dn(P * P, 0.0L);
  for (int j = 0; j < P; ++j) {
    long double diag = 0.0L;
    for (int i = 0; i < P; ++i) {
      if (i == j) continue;
      Dn[j * P + i] = (bw[i] / bw[j]) / ((long double)xn[j] - xn[i]);
      diag -= Dn[j * P + i];
    }
    Dn[j * P + j] = diag;
  }
  B.assign(Q * P, 0.0);
  D.assign(Q * P, 0.0);
  for (int q = 0; q < Q; ++q) {
    std::vector<long double> l(P, 0.0L);
    int hit = -1;
    for (int j = 0; j < P; ++j)
      if ((long double)xq[q] == (long double)xn[j]) hit = j;
    if (hit >= 0) {
      l[hit] = 1.0L;
    } else {
      long double den = 0.0L;
      for (int j = 0; j < P; ++j) den += bw[j] / ((long double)xq[q] - xn[j]);
      for (int j = 0; j < P; ++j) l[j] = (bw[j] / ((long double)xq[q] - xn[j])) / den;
    }
    for (int i = 0; i < P; ++i) {
      B[q * P + i] = (double)l[i];
      long double d = 0.0L;
      for (int j = 0; j < P; ++j) d += l[j] * Dn[j * P + i];
      D[q * P + i] = (double)d;
    }
  }
}

}  // namespace pfmf
