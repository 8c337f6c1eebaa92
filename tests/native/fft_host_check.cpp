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

#define RUN(P)                                                                          \
  {                                                                                     \
    double e1 = check_fft_reg<P, -1>(), e2 = check_fft_reg<P, +1>(), e3 = check_twiddles<P>(); \
    std::printf("P=%d fwd=%.3e inv=%.3e tw=%.3e\n", P, e1, e2, e3);                        \
    worst = std::fmax(worst, std::fmax(std::fmax(e1, e2) / std::sqrt((double)P), e3));  \
  }

int main() {
  double worst = 0;
  RUN(8) RUN(12) RUN(16) RUN(24) RUN(32) RUN(36) RUN(48) RUN(64) RUN(72) RUN(96)
  std::printf("worst %.3e\n", worst);
  return worst < 1e-14 ? 0 : 1;
}
