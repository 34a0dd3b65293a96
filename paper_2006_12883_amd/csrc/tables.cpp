// Right-Radau tables in long double (see tables.hpp for the definitions).
#include "tables.hpp"

#include <cmath>

namespace stmg {

namespace {

// Legendre P_n(x) and its derivative by the three-term recurrence.
void legendre(int n, long double x, long double* p, long double* dp) {
  if (n == 0) { *p = 1.0L; *dp = 0.0L; return; }
  long double p0 = 1.0L, p1 = x;
  for (int k = 1; k < n; ++k) {
    long double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  *p = p1;
  // (1 - x^2) P_n' = n (P_{n-1} - x P_n); not used at x = +-1
  *dp = (std::fabs(1.0L - x * x) > 1e-30L) ? n * (p0 - x * p1) / (1.0L - x * x) : 0.0L;
}

// g(t) = P_M(2t-1) - P_{M-1}(2t-1): its roots are the right Radau nodes.
long double radau_poly(int M, long double t) {
  long double a, da, b, db;
  legendre(M, 2.0L * t - 1.0L, &a, &da);
  legendre(M - 1, 2.0L * t - 1.0L, &b, &db);
  return a - b;
}

// Gauss-Legendre rule with K points on [-1, 1] (Newton on P_K).
void gauss_legendre(int K, long double* x, long double* w) {
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < K; ++i) {
    long double z = std::cos(pi * (i + 0.75L) / (K + 0.5L));
    for (int it = 0; it < 100; ++it) {
      long double p, dp;
      legendre(K, z, &p, &dp);
      long double dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    long double p, dp;
    legendre(K, z, &p, &dp);
    x[i] = z;
    w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
  }
}

long double lagrange(const long double* c, int M, int j, long double t) {
  long double v = 1.0L;
  for (int k = 0; k < M; ++k)
    if (k != j) v *= (t - c[k]) / (c[j] - c[k]);
  return v;
}

}  // namespace

bool invert_ld(std::vector<long double>& a, int n) {
  std::vector<long double> inv(static_cast<size_t>(n) * n, 0.0L);
  for (int i = 0; i < n; ++i) inv[static_cast<size_t>(i) * n + i] = 1.0L;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    long double best = std::fabs(a[static_cast<size_t>(col) * n + col]);
    for (int r = col + 1; r < n; ++r) {
      long double v = std::fabs(a[static_cast<size_t>(r) * n + col]);
      if (v > best) { best = v; piv = r; }
    }
    if (!(best > 0.0L)) return false;
    if (piv != col) {
      for (int k = 0; k < n; ++k) {
        std::swap(a[static_cast<size_t>(piv) * n + k], a[static_cast<size_t>(col) * n + k]);
        std::swap(inv[static_cast<size_t>(piv) * n + k], inv[static_cast<size_t>(col) * n + k]);
      }
    }
    long double d = a[static_cast<size_t>(col) * n + col];
    for (int k = 0; k < n; ++k) {
      a[static_cast<size_t>(col) * n + k] /= d;
      inv[static_cast<size_t>(col) * n + k] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      long double f = a[static_cast<size_t>(r) * n + col];
      if (f == 0.0L) continue;
      for (int k = 0; k < n; ++k) {
        a[static_cast<size_t>(r) * n + k] -= f * a[static_cast<size_t>(col) * n + k];
        inv[static_cast<size_t>(r) * n + k] -= f * inv[static_cast<size_t>(col) * n + k];
      }
    }
  }
  a.swap(inv);
  return true;
}

bool radau_tables(int M, RadauTables* t) {
  if (M < 1 || M > 8) return false;
  t->M = M;
  // Nodes: scan (0, 1) for sign changes of the Radau polynomial, bisect, then
  // polish with a few secant steps; the last node is exactly 1.
  int found = 0;
  const int S = 20000;
  long double prev_t = 0.0L, prev_g = radau_poly(M, 0.0L);
  for (int s = 1; s <= S && found < M - 1; ++s) {
    long double tt = static_cast<long double>(s) / S;
    if (s == S) break;
    long double g = radau_poly(M, tt);
    if ((g < 0) != (prev_g < 0)) {
      long double lo = prev_t, hi = tt, glo = prev_g;
      for (int it = 0; it < 200; ++it) {
        long double mid = 0.5L * (lo + hi);
        long double gm = radau_poly(M, mid);
        if ((gm < 0) == (glo < 0)) { lo = mid; glo = gm; } else { hi = mid; }
      }
      t->c[found++] = 0.5L * (lo + hi);
    }
    prev_t = tt;
    prev_g = g;
  }
  if (found != M - 1) return false;
  t->c[M - 1] = 1.0L;

  // Q[m][j] = int_0^{c_m} l_j(s) ds with an exact Gauss-Legendre rule.
  long double gx[12], gw[12];
  gauss_legendre(12, gx, gw);
  for (int m = 0; m < M; ++m)
    for (int j = 0; j < M; ++j) {
      long double acc = 0.0L;
      for (int q = 0; q < 12; ++q) {
        long double s = 0.5L * t->c[m] * (gx[q] + 1.0L);
        acc += 0.5L * t->c[m] * gw[q] * lagrange(t->c, M, j, s);
      }
      t->Q[m][j] = acc;
    }
  for (int j = 0; j < M; ++j) t->b[j] = t->Q[M - 1][j];

  std::vector<long double> Qi(static_cast<size_t>(M) * M);
  for (int i = 0; i < M; ++i)
    for (int j = 0; j < M; ++j) Qi[static_cast<size_t>(i) * M + j] = t->Q[i][j];
  if (!invert_ld(Qi, M)) return false;
  for (int i = 0; i < M; ++i) {
    long double s = 0.0L;
    for (int j = 0; j < M; ++j) {
      t->Kq[i][j] = t->b[i] * Qi[static_cast<size_t>(i) * M + j];
      s += t->Kq[i][j];
    }
    t->l0[i] = s;
  }
  return true;
}

}  // namespace stmg
