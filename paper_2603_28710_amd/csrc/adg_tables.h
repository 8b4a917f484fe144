// adg_tables.h — the 1D operators of the nodal DG discretisation (Sec. 2.1),
// evaluated at compile time for P = degree + 1 Gauss-Lobatto-Legendre nodes
// and Q = P + 1 Gauss-Legendre points, so kernels see them as constants and
// the host fills its run-time table from the same numbers.
#pragma once

namespace adg {
namespace ops {

struct Leg {
  double p, dp;
};

// P_n(x) by the three-term recurrence and P_n'(x) from
// (x^2 - 1) P_n' = n (x P_n - P_{n-1}) (|x| < 1)
constexpr Leg legendre(int n, double x) {
  if (n == 0) return {1.0, 0.0};
  double p0 = 1.0, p1 = x;
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  return {p1, n * (x * p1 - p0) / (x * x - 1.0)};
}

constexpr double cabs(double x) { return x < 0 ? -x : x; }

// the root of f in (lo, hi) where f changes sign, by bisection to the last bit
template <class F>
constexpr double bisect(F f, double lo, double hi) {
  double flo = f(lo), fhi = f(hi);
  for (int it = 0; it < 2000; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    const double fm = f(mid);
    if (fm == 0.0) return mid;
    if ((fm < 0) == (flo < 0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
      fhi = fm;
    }
  }
  return cabs(flo) <= cabs(fhi) ? lo : hi;
}

// the m roots in (-1, 1) of f, located by sign changes on a fine grid
template <class F>
constexpr void roots(F f, int m, double* x) {
  constexpr int kGrid = 1024;
  int found = 0;
  double a = -1.0 + 1.0 / kGrid, fa = f(a);
  for (int i = 1; i < 2 * kGrid - 1 && found < m; ++i) {
    const double b = -1.0 + (i + 1.0) / kGrid, fb = f(b);
    if (fa == 0.0) {
      x[found++] = a;
    } else if (fb != 0.0 && (fa < 0) != (fb < 0)) {
      x[found++] = bisect(f, a, b);
    }
    a = b;
    fa = fb;
  }
}

template <int P>
struct Ops {
  static constexpr int Q = P + 1;
  double xg[Q], wg[Q];  // Gauss-Legendre points and weights
  double xl[P], wl[P];  // Gauss-Lobatto-Legendre nodes and weights
  double B[Q][P];       // B[q][j] = l_j(x_q), GLL Lagrange basis at the Gauss points
  double D[Q][Q];       // D[q][r] = g_r'(x_q), g the Gauss-point Lagrange basis
  double MI[P][P];      // inverse of the 1D mass matrix M1[i][j] = sum_q w_q B[q][i] B[q][j]
  double BTM[P][Q];     // MI B^T
  double BW[P][Q];      // MI B^T W
  double GW[P][Q];      // MI B^T D^T W
  double MC[2][P];      // columns 0 and P-1 of MI
};

template <int P>
constexpr Ops<P> make_ops() {
  constexpr int Q = P + 1, N = P - 1;
  Ops<P> o{};
  // Gauss: zeros of P_Q, weights 2 / ((1 - x^2) P_Q'(x)^2)
  roots([](double x) { return legendre(Q, x).p; }, Q, o.xg);
  for (int q = 0; q < Q; ++q) {
    const double d = legendre(Q, o.xg[q]).dp;
    o.wg[q] = 2.0 / ((1.0 - o.xg[q] * o.xg[q]) * d * d);
  }
  // GLL: -1, the zeros of P_N', +1; weights 2 / (N (N+1) P_N(x)^2)
  o.xl[0] = -1.0;
  o.xl[N] = 1.0;
  if (N >= 2) {
    double in[P] = {};
    roots([](double x) { return legendre(N, x).dp; }, N - 1, in);
    for (int i = 1; i < N; ++i) o.xl[i] = in[i - 1];
  }
  for (int i = 0; i < P; ++i) {
    double pn = 1.0;
    if (o.xl[i] == 1.0 || o.xl[i] == -1.0)
      pn = (N % 2 == 1 && o.xl[i] < 0) ? -1.0 : 1.0;
    else
      pn = legendre(N, o.xl[i]).p;
    o.wl[i] = 2.0 / (N * (N + 1.0) * pn * pn);
  }
  // Lagrange basis on the GLL nodes at the Gauss points (product form)
  for (int q = 0; q < Q; ++q)
    for (int j = 0; j < P; ++j) {
      double l = 1.0;
      for (int m = 0; m < P; ++m)
        if (m != j) l *= (o.xg[q] - o.xl[m]) / (o.xl[j] - o.xl[m]);
      o.B[q][j] = l;
    }
  // collocation derivative on the Gauss points (barycentric weights)
  double lam[Q] = {};
  for (int r = 0; r < Q; ++r) {
    lam[r] = 1.0;
    for (int m = 0; m < Q; ++m)
      if (m != r) lam[r] /= (o.xg[r] - o.xg[m]);
  }
  for (int q = 0; q < Q; ++q) {
    double diag = 0.0;
    for (int r = 0; r < Q; ++r) {
      if (r == q) continue;
      o.D[q][r] = (lam[r] / lam[q]) / (o.xg[q] - o.xg[r]);
      diag -= o.D[q][r];
    }
    o.D[q][q] = diag;
  }
  // mass matrix and its inverse (Gauss-Jordan with partial pivoting)
  double a[P][2 * P] = {};
  for (int i = 0; i < P; ++i) {
    for (int j = 0; j < P; ++j) {
      double m = 0.0;
      for (int q = 0; q < Q; ++q) m += o.wg[q] * o.B[q][i] * o.B[q][j];
      a[i][j] = m;
    }
    a[i][P + i] = 1.0;
  }
  for (int c = 0; c < P; ++c) {
    int piv = c;
    for (int r = c + 1; r < P; ++r)
      if (cabs(a[r][c]) > cabs(a[piv][c])) piv = r;
    for (int k = 0; k < 2 * P; ++k) {
      const double t = a[c][k];
      a[c][k] = a[piv][k];
      a[piv][k] = t;
    }
    const double d = a[c][c];
    for (int k = 0; k < 2 * P; ++k) a[c][k] /= d;
    for (int r = 0; r < P; ++r) {
      if (r == c) continue;
      const double f = a[r][c];
      for (int k = 0; k < 2 * P; ++k) a[r][k] -= f * a[c][k];
    }
  }
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < P; ++j) o.MI[i][j] = a[i][P + j];
  for (int i = 0; i < P; ++i)
    for (int q = 0; q < Q; ++q) {
      double b = 0.0;
      for (int j = 0; j < P; ++j) b += o.MI[i][j] * o.B[q][j];
      o.BTM[i][q] = b;
      o.BW[i][q] = b * o.wg[q];
    }
  for (int i = 0; i < P; ++i)
    for (int q = 0; q < Q; ++q) {
      double g = 0.0;
      for (int r = 0; r < Q; ++r) g += o.BTM[i][r] * o.D[q][r];
      o.GW[i][q] = g * o.wg[q];
    }
  for (int i = 0; i < P; ++i) {
    o.MC[0][i] = o.MI[i][0];
    o.MC[1][i] = o.MI[i][P - 1];
  }
  return o;
}

template <int P>
inline constexpr Ops<P> kOps = make_ops<P>();

// the entries a sweep over Gauss index q reads at run time, contiguous per q
// (one wide scalar load): B[q][j], BW[j][q], GW[j][q] for j < P
template <int P>
struct alignas(64) RowOps {
  double r[P + 1][3][P];
};

template <int P>
constexpr RowOps<P> make_rowops() {
  RowOps<P> t{};
  for (int q = 0; q <= P; ++q)
    for (int j = 0; j < P; ++j) {
      t.r[q][0][j] = kOps<P>.B[q][j];
      t.r[q][1][j] = kOps<P>.BW[j][q];
      t.r[q][2][j] = kOps<P>.GW[j][q];
    }
  return t;
}

template <int P>
inline constexpr RowOps<P> kRowOps = make_rowops<P>();

}  // namespace ops
}  // namespace adg
