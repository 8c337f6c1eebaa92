// Host-side quadrature rules of the plan (Section 4, eq. approxG, and the
// t-integral of the angular weight F, eq. FF):
//   * Gauss-Legendre nodes in |q| on [0, R]: Newton on the Legendre recurrence
//     in long double;
//   * Gauss-Jacobi nodes for \int_0^1 t^{-s} (1-t)^{-r} g(t) dt: eigenvalues of
//     the Jacobi matrix by Sturm bisection (Golub-Welsch), polished by Newton
//     on the Jacobi recurrence in long double, weights from the classical
//     closed form;
//   * Lebedev rules on S^2 from the generated table, split into antipodal
//     halves (the rules are centrally symmetric with equal weights).
#include "quadrature.hpp"

#include <cmath>
#include <vector>

namespace bzq {

namespace {
#include "lebedev_rules.inc"
}

void gauss_legendre(int n, double R, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double z = cosl(pi * (i + 0.75L) / (n + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    {  // derivative at the converged node
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
    }
    // nodes in increasing order on [0, R]
    const long double wz = 2.0L / ((1 - z * z) * dp * dp);
    x[n - 1 - i] = (double)(0.5L * R * (1.0L + z));
    w[n - 1 - i] = (double)(0.5L * R * wz);
  }
}

namespace {
// P_n^{(a,b)}(x) and P_{n-1}^{(a,b)}(x) by the three-term recurrence
void jacobi_eval(int n, long double a, long double b, long double x, long double& pn,
                 long double& pm) {
  long double p0 = 1;
  long double p1 = (a - b) / 2 + (a + b + 2) * x / 2;
  if (n == 0) { pn = p0; pm = 0; return; }
  if (n == 1) { pn = p1; pm = p0; return; }
  for (int k = 2; k <= n; ++k) {
    long double c = 2 * k + a + b;
    long double a1 = 2 * k * (k + a + b) * (c - 2);
    long double a2 = (c - 1) * (a * a - b * b);
    long double a3 = (c - 2) * (c - 1) * c;
    long double a4 = 2 * (k + a - 1) * (k + b - 1) * c;
    long double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pm = p0;
}

// number of eigenvalues of the symmetric tridiagonal (d, e2 = off-diagonal^2) below x
int sturm_count(const std::vector<long double>& d, const std::vector<long double>& e2, long double x) {
  int cnt = 0;
  long double q = 1;
  for (size_t i = 0; i < d.size(); ++i) {
    q = d[i] - x - (i ? e2[i] / q : 0.0L);
    if (q == 0) q = -1e-30L;
    if (q < 0) ++cnt;
  }
  return cnt;
}
}  // namespace

bool gauss_jacobi01(int n, double s, double r, std::vector<double>& t, std::vector<double>& w) {
  // weight (1-u)^alpha (1+u)^beta on [-1, 1], alpha = -r, beta = -s
  const long double a = -r, b = -s;
  if (n < 1 || !(a > -1) || !(b > -1)) return false;
  // monic Jacobi recurrence: diagonal d_k, squared off-diagonal e2_k
  std::vector<long double> d(n), e2(n, 0.0L);
  for (int k = 0; k < n; ++k) {
    long double c = 2 * k + a + b;
    if (k == 0)
      d[k] = (b - a) / (a + b + 2);
    else
      d[k] = (b * b - a * a) / (c * (c + 2));
    if (k >= 1) {
      if (k == 1)
        e2[k] = 4 * (1 + a) * (1 + b) / ((2 + a + b) * (2 + a + b) * (3 + a + b));
      else
        e2[k] = 4 * k * (k + a) * (k + b) * (k + a + b) / (c * c * (c + 1) * (c - 1));
    }
  }
  const long double logc = lgammal(n + a + 1) + lgammal(n + b + 1) - lgammal(n + a + b + 1) -
                           lgammal((long double)n + 1);
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    // i-th smallest eigenvalue by bisection on [-1, 1]
    long double lo = -1, hi = 1;
    for (int it = 0; it < 80; ++it) {
      long double mid = 0.5L * (lo + hi);
      if (sturm_count(d, e2, mid) > i) hi = mid; else lo = mid;
    }
    long double x = 0.5L * (lo + hi), pn, pm;
    for (int it = 0; it < 8; ++it) {
      jacobi_eval(n, a, b, x, pn, pm);
      long double c = 2 * n + a + b;
      long double dp = (n * ((a - b) - c * x) * pn + 2 * (n + a) * (n + b) * pm) / (c * (1 - x * x));
      long double dx = pn / dp;
      x -= dx;
      if (fabsl(dx) < 1e-19L) break;
    }
    jacobi_eval(n, a, b, x, pn, pm);
    long double c = 2 * n + a + b;
    long double dp = (n * ((a - b) - c * x) * pn + 2 * (n + a) * (n + b) * pm) / (c * (1 - x * x));
    // on [0, 1]: t = (u + 1)/2 and the weight constant loses its 2^{a+b+1}
    long double wu = expl(logc) / ((1 - x * x) * dp * dp);
    t[i] = (double)(0.5L * (x + 1));
    w[i] = (double)wu;
  }
  return true;
}

void gauss_laguerre(int n, std::vector<long double>& u, std::vector<long double>& w) {
  // Jacobi matrix of the Laguerre polynomials: diagonal 2k+1, off-diagonal k
  std::vector<long double> d(n), e2(n, 0.0L);
  for (int k = 0; k < n; ++k) {
    d[k] = 2.0L * k + 1.0L;
    if (k >= 1) e2[k] = (long double)k * k;
  }
  u.assign(n, 0.0L);
  w.assign(n, 0.0L);
  const long double hi0 = 4.0L * n + 4.0L;   // every node lies below 4n + 2
  for (int i = 0; i < n; ++i) {
    long double lo = 0, hi = hi0;
    for (int it = 0; it < 90; ++it) {
      const long double mid = 0.5L * (lo + hi);
      if (sturm_count(d, e2, mid) > i) hi = mid; else lo = mid;
    }
    long double x = 0.5L * (lo + hi);
    // Newton on L_n, with L_{n-1} for the derivative: x L_n' = n (L_n - L_{n-1})
    long double ln = 0, lm = 0;
    for (int it = 0; it < 6; ++it) {
      long double p0 = 1, p1 = 1 - x;
      for (int k = 1; k < n; ++k) {
        const long double p2 = ((2 * k + 1 - x) * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
      }
      ln = n == 0 ? 1 : p1;
      lm = n == 0 ? 0 : p0;
      const long double dp = n * (ln - lm) / x;
      const long double dx = ln / dp;
      x -= dx;
      if (fabsl(dx) < 1e-21L * (1 + x)) break;
    }
    // w = x / ((n+1)^2 L_{n+1}(x)^2)
    long double p0 = 1, p1 = 1 - x;
    for (int k = 1; k <= n; ++k) {
      const long double p2 = ((2 * k + 1 - x) * p1 - k * p0) / (k + 1);
      p0 = p1;
      p1 = p2;
    }
    u[i] = x;
    w[i] = x / ((long double)(n + 1) * (n + 1) * p1 * p1);
  }
}

bool debye_rule(double theta_cut, std::vector<double>& t, std::vector<double>& w) {
  const long double pi = 3.141592653589793238462643383279502884L;
  if (!(theta_cut >= 0.0 && theta_cut < (double)(pi / 3))) return false;
  t.clear();
  w.clear();
  auto wlog = [](long double x) { return fabsl(logl(2.0L * sqrtl(x))) / sqrtl(1.0L - x); };
  // [1/4, 1]: t = 1/4 + 3s/4, (1-t)^{-1/2} = (3/4)^{-1/2} (1-s)^{-1/2}, dt = 3/4 ds
  std::vector<double> sj, wj;
  if (!gauss_jacobi01(64, 0.0, 0.5, sj, wj)) return false;
  for (size_t i = 0; i < sj.size(); ++i) {
    const long double ti = 0.25L + 0.75L * sj[i];
    t.push_back((double)ti);
    w.push_back((double)(wj[i] * sqrtl(0.75L) * logl(2.0L * sqrtl(ti))));
  }
  // Gauss-Legendre panels [a, b] with the whole weight in the integrand
  auto panel = [&](long double a, long double b, int n) {
    std::vector<double> x, g;
    gauss_legendre(n, 1.0, x, g);          // on [0, 1]
    for (int i = 0; i < n; ++i) {
      const long double ti = a + (b - a) * x[i];
      t.push_back((double)ti);
      w.push_back((double)((b - a) * g[i] * wlog(ti)));
    }
  };
  const long double tc = powl(sinl(0.5L * theta_cut), 2), t0 = 1e-6L;
  long double hi = 0.25L;
  for (int k = 0;; ++k) {
    const long double lo = hi / 8.0L;
    const int n = k == 0 ? 32 : k == 1 ? 24 : 16;
    if (theta_cut > 0.0 && lo <= tc) {
      panel(tc, hi, n);
      break;
    }
    if (lo <= t0) {
      panel(t0, hi, n);
      if (theta_cut == 0.0) {
        // [0, t0]: t = t0 e^{-u}, |log(2 sqrt t)| = (u + log(1/(4 t0)))/2, dt = t du
        std::vector<long double> u, om;
        gauss_laguerre(20, u, om);
        for (int i = 0; i < 20; ++i) {
          const long double ti = t0 * expl(-u[i]);
          t.push_back((double)ti);
          w.push_back((double)(om[i] * t0 * (u[i] + logl(1.0L / (4.0L * t0))) / 2.0L / sqrtl(1.0L - ti)));
        }
      }
      break;
    }
    panel(lo, hi, n);
    hi = lo;
  }
  return true;
}

bool lebedev_rule(int M, std::vector<double>& xyzw) {
  for (int i = 0; i < kLebedevCount; ++i) {
    if (kLebedevIndex[i][0] == M) {
      xyzw.assign(4 * M, 0.0);
      const int o = kLebedevIndex[i][2];
      for (int j = 0; j < M; ++j) {
        long double x = kLebedevRows[o + j][0], y = kLebedevRows[o + j][1], z = kLebedevRows[o + j][2];
        long double nrm = sqrtl(x * x + y * y + z * z);
        xyzw[4 * j + 0] = (double)(x / nrm);
        xyzw[4 * j + 1] = (double)(y / nrm);
        xyzw[4 * j + 2] = (double)(z / nrm);
        xyzw[4 * j + 3] = kLebedevRows[o + j][3];
      }
      return true;
    }
  }
  return false;
}

int lebedev_half(const std::vector<double>& xyzw, std::vector<double>& half) {
  const int M = (int)(xyzw.size() / 4);
  half.clear();
  int matched = 0;
  for (int j = 0; j < M; ++j) {
    const double* p = &xyzw[4 * j];
    double lead = std::fabs(p[0]) > 1e-12 ? p[0] : (std::fabs(p[1]) > 1e-12 ? p[1] : p[2]);
    if (lead <= 0) continue;
    // antipode must exist with the same weight
    bool ok = false;
    for (int k = 0; k < M; ++k) {
      const double* q = &xyzw[4 * k];
      if (std::fabs(p[0] + q[0]) < 1e-13 && std::fabs(p[1] + q[1]) < 1e-13 &&
          std::fabs(p[2] + q[2]) < 1e-13 && std::fabs(p[3] - q[3]) <= 1e-14 * std::fabs(p[3])) {
        ok = true;
        break;
      }
    }
    if (!ok) return -1;
    half.insert(half.end(), p, p + 4);
    ++matched;
  }
  return 2 * matched == M ? matched : -1;
}

}  // namespace bzq
