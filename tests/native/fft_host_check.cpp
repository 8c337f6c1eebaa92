// Host-side check of the device FFT building blocks (compiled for the host
// only): every small DFT and every register FFT length against a direct
// long-double DFT, both signs, and the compile-time twiddles against libm.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>

#include "fft.hpp"

using namespace bzq;
typedef std::complex<long double> C;

template <int P, int SIGN>
double check_fft_reg() {
  std::mt19937_64 g(P * 7 + SIGN + 3);
  std::uniform_real_distribution<double> u(-1, 1);
  cx<double> x[P];
  C ref[P];
  for (int i = 0; i < P; ++i) x[i] = {u(g), u(g)};
  for (int k = 0; k < P; ++k) {
    C acc = 0;
    for (int n = 0; n < P; ++n) {
      long double a = SIGN * 2.0L * 3.141592653589793238462643383279502884L * ((long double)n * k) / P;
      acc += C(x[n].x, x[n].y) * C(cosl(a), sinl(a));
    }
    ref[k] = acc;
  }
  fft_reg<P, SIGN>(x);
  double err = 0;
  for (int k = 0; k < P; ++k) err = std::fmax(err, (double)std::abs(C(x[k].x, x[k].y) - ref[k]));
  return err;
}

template <int P>
double check_twiddles() {
  constexpr TwiddleTable<P> tw{};
  double err = 0;
  for (int m = 0; m < P; ++m) {
    long double a = 2.0L * 3.141592653589793238462643383279502884L * m / P;
    err = std::fmax(err, std::fabs((double)(tw.c[m] - cosl(a))));
    err = std::fmax(err, std::fabs((double)(tw.s[m] - sinl(a))));
  }
  return err;
}

// half transforms by one decimation step in frequency: outputs of parity PAR
template <int P, int SIGN, int PAR>
double check_half() {
  std::mt19937_64 g(P * 11 + SIGN * 3 + PAR);
  std::uniform_real_distribution<double> ud(-1, 1);
  cx<double> x[P];
  for (int i = 0; i < P; ++i) x[i] = {ud(g), ud(g)};
  cx<double> u[P / 2];
  dft_half_dif<P, SIGN, PAR>([&](int n) { return x[n]; }, u);
  double err = 0;
  for (int j = 0; j < P / 2; ++j) {
    const int k = 2 * j + PAR;
    C acc = 0;
    for (int n = 0; n < P; ++n) {
      long double a = SIGN * 2.0L * 3.141592653589793238462643383279502884L * ((long double)n * k) / P;
      acc += C(x[n].x, x[n].y) * C(cosl(a), sinl(a));
    }
    err = std::fmax(err, (double)std::abs(C(u[j].x, u[j].y) - acc));
  }
  return err;
}

// forward transform assembled from its two parities by one decimation step in
// time, with the exchange of halves used by the plane kernel: parity 0 holds
// E = DFT_Q(x[2j]), parity 1 holds w^{-k} O[k], O = DFT_Q(x[2j+1]); after the
// exchange u0[i] = X[i], u0[Q/2+i] = X[Q+i], u1[i] = X[Q/2+i], u1[Q/2+i] = X[Q+Q/2+i]
template <int P>
double check_dit_exchange() {
  constexpr int Q = P / 2, QH = Q / 2;
  std::mt19937_64 g(P * 13 + 5);
  std::uniform_real_distribution<double> ud(-1, 1);
  cx<double> x[P], u0[Q], u1[Q];
  for (int i = 0; i < P; ++i) x[i] = {ud(g), ud(g)};
  for (int j = 0; j < Q; ++j) { u0[j] = x[2 * j]; u1[j] = x[2 * j + 1]; }
  fft_reg<Q, -1>(u0);
  fft_reg<Q, -1>(u1);
  for (int k = 1; k < Q; ++k) u1[k] = twiddle_mul<P, -1>(u1[k], k);
  cx<double> xa[QH], xb[QH];
  for (int i = 0; i < QH; ++i) { xa[i] = u0[QH + i]; xb[i] = u1[i]; }
  for (int i = 0; i < QH; ++i) {
    const cx<double> e0 = u0[i], t0 = xb[i];
    u0[i] = cadd(e0, t0); u0[QH + i] = csub(e0, t0);
    const cx<double> e1 = xa[i], t1 = u1[QH + i];
    u1[i] = cadd(e1, t1); u1[QH + i] = csub(e1, t1);
  }
  double err = 0;
  for (int k = 0; k < P; ++k) {
    C acc = 0;
    for (int n = 0; n < P; ++n) {
      long double a = -2.0L * 3.141592653589793238462643383279502884L * ((long double)n * k) / P;
      acc += C(x[n].x, x[n].y) * C(cosl(a), sinl(a));
    }
    const int half = k < Q ? 0 : 1, kk = k % Q;
    const cx<double> got = kk < QH ? (half ? u0[QH + kk] : u0[kk]) : (half ? u1[QH + kk - QH] : u1[kk - QH]);
    err = std::fmax(err, (double)std::abs(C(got.x, got.y) - acc));
  }
  return err;
}

// quarter transforms by one radix-4 decimation step in frequency: outputs 4j + R
template <int P, int SIGN, int R>
double check_quarter() {
  std::mt19937_64 g(P * 17 + SIGN * 5 + R);
  std::uniform_real_distribution<double> ud(-1, 1);
  cx<double> x[P];
  for (int i = 0; i < P; ++i) x[i] = {ud(g), ud(g)};
  cx<double> u[P / 4];
  dft_quarter_dif<P, SIGN, R>([&](int n) { return x[n]; }, u);
  double err = 0;
  for (int j = 0; j < P / 4; ++j) {
    const int k = 4 * j + R;
    C acc = 0;
    for (int n = 0; n < P; ++n) {
      long double a = SIGN * 2.0L * 3.141592653589793238462643383279502884L * ((long double)n * k) / P;
      acc += C(x[n].x, x[n].y) * C(cosl(a), sinl(a));
    }
    err = std::fmax(err, (double)std::abs(C(u[j].x, u[j].y) - acc));
  }
  return err;
}

#define QUARTER(P)                                                                                    \
  {                                                                                                   \
    double e = 0;                                                                                     \
    e = std::fmax(e, std::fmax(check_quarter<P, -1, 0>(), check_quarter<P, -1, 1>()));              \
    e = std::fmax(e, std::fmax(check_quarter<P, -1, 2>(), check_quarter<P, -1, 3>()));              \
    e = std::fmax(e, std::fmax(check_quarter<P, +1, 0>(), check_quarter<P, +1, 1>()));              \
    e = std::fmax(e, std::fmax(check_quarter<P, +1, 2>(), check_quarter<P, +1, 3>()));              \
    std::printf("P=%d quarter=%.3e\n", P, e);                                                       \
    worst = std::fmax(worst, e / std::sqrt((double)P));                                               \
  }

#define HALF(P)                                                                                       \
  {                                                                                                   \
    double e = std::fmax(std::fmax(check_half<P, -1, 0>(), check_half<P, -1, 1>()),                  \
                         std::fmax(check_half<P, +1, 0>(), check_half<P, +1, 1>()));                  \
    double d = check_dit_exchange<P>();                                                               \
    std::printf("P=%d half=%.3e dit-exchange=%.3e\n", P, e, d);                                       \
    worst = std::fmax(worst, std::fmax(e, d) / std::sqrt((double)P));                                 \
  }

#define RUN(P)                                                                          \
  {                                                                                     \
    double e1 = check_fft_reg<P, -1>(), e2 = check_fft_reg<P, +1>(), e3 = check_twiddles<P>(); \
    std::printf("P=%d fwd=%.3e inv=%.3e tw=%.3e\n", P, e1, e2, e3);                        \
    worst = std::fmax(worst, std::fmax(std::fmax(e1, e2) / std::sqrt((double)P), e3));  \
  }

int main() {
  double worst = 0;
  RUN(8) RUN(12) RUN(16) RUN(24) RUN(32) RUN(36) RUN(48) RUN(64) RUN(72) RUN(96)
  HALF(48) HALF(72) HALF(96)
  QUARTER(32) QUARTER(48) QUARTER(96)
  std::printf("worst %.3e\n", worst);
  return worst < 1e-14 ? 0 : 1;
}
