// C ABI of the two-dimensional operator: plans and evaluation.
//
// The 2-D Galerkin system of Section 2 with d = 2: radial Gauss-Legendre rule
// on [0, R], the midpoint rule on the circle (the paper's choice for its 2-D
// tests, Section 5.2), the exact angular weight of eq. FF2D1 by Gauss-Jacobi
// quadrature in t = sin^2(th/2), antipodal circle points paired as in 3-D.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/bzq.h"
#include "kernels.hpp"
#include "kernels2d.hpp"
#include "plan.hpp"
#include "quadrature.hpp"

namespace bzq {
namespace {
const long double kPi2 = 3.141592653589793238462643383279502884L;
}
}  // namespace bzq

struct bzq_plan2d_s {
  int N = 0, P = 0, nh = 0, npairs = 0, npt = 0, S = 0;
  bool fp32 = false;
  void* V = nullptr;
  double* ph = nullptr;
  double* cp = nullptr;
  void* tw = nullptr;
  void* fc = nullptr;
  void* fgrid = nullptr;
  double* Qpart = nullptr;
  double* fin = nullptr;  // 16 chunk sums of the partials
  double* q1 = nullptr;   // stage results and stage argument of the time steps (N^2 complex each)
  double* q2 = nullptr;
  double* fs = nullptr;
  bzq::DeviceArena mem;
};

using namespace bzq;

namespace {
hipError_t collide(bzq_plan2d p, const double* f_hat, double* Q_hat, hipStream_t st) {
  return launch_collision2d(f_hat, Q_hat, p->fc, p->fgrid, p->V, p->ph, p->cp, p->tw, p->Qpart, p->fin, p->N,
                            p->P, p->npt, p->S, p->fp32, st);
}
}  // namespace

extern "C" {

bzq_status bzq_plan2d_create(bzq_plan2d* out, int N, double L, double R, double gamma, double b_c, double b_s,
                             double b_r, int n_jacobi, int N_rho, int N_sigma, int precision, void* stream) {
  if (!out) return fail(BZQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (N < 8 || (N & 1)) return fail(BZQ_EINVAL, "N must be even and >= 8");
  if (!(L > 0) || !std::isfinite(L)) return fail(BZQ_EINVAL, "L must be > 0");
  if (!(R > 0) || !std::isfinite(R)) return fail(BZQ_EINVAL, "R must be > 0");
  if (!(gamma > -2.0 && gamma <= 1.0)) return fail(BZQ_EINVAL, "gamma must lie in (-2, 1]");
  if (!(b_c > 0) || !std::isfinite(b_c)) return fail(BZQ_EINVAL, "kernel constant c must be > 0");
  if (!(b_s >= -1.0 && b_s < 0.5)) return fail(BZQ_EINVAL, "s must lie in [-1, 1/2) in 2-D");
  if (!(b_r > -1.0 && b_r < 0.5)) return fail(BZQ_EINVAL, "r must lie in (-1, 1/2) in 2-D");
  if (n_jacobi < 8 || n_jacobi > 256) return fail(BZQ_EINVAL, "n_jacobi must lie in [8, 256]");
  if (N_rho < 1 || N_rho > 4096) return fail(BZQ_EINVAL, "N_rho must lie in [1, 4096]");
  if (N_sigma < 2 || (N_sigma & 1) || N_sigma > 4096) return fail(BZQ_EINVAL, "N_sigma must be even, 2..4096");
  if (precision != BZQ_FP64 && precision != BZQ_FP32_ACC64) return fail(BZQ_EINVAL, "unknown precision");
  if (!(N == 8 || N == 16 || N == 24 || N == 32 || N == 48 || N == 64))
    return fail(BZQ_EUNSUPPORTED, "no FFT schedule for this N (supported: 8 16 24 32 48 64)");
  hipStream_t st = (hipStream_t)stream;
  auto* p = new bzq_plan2d_s();
  p->N = N;
  p->P = 3 * N / 2;
  const int n1 = N - 1, P = p->P, PL = 2 * N - 3;
  p->nh = (n1 * n1 + 1) / 2;
  p->fp32 = precision == BZQ_FP32_ACC64;
  const size_t esz = p->fp32 ? 4 : 8;
  std::vector<double> rho, wr, gt, gw;
  gauss_legendre(N_rho, R, rho, wr);
  if (!gauss_jacobi01(n_jacobi, b_s + 0.5, b_r + 0.5, gt, gw)) {
    delete p;
    return fail(BZQ_EINVAL, "Gauss-Jacobi rule failed");
  }
  const int half = N_sigma / 2, nreal = N_rho * half;
  p->npairs = nreal + (nreal & 1);
  p->npt = p->npairs / 2;
  std::vector<double> pd((size_t)p->npairs * 4, 0.0), cp(p->npairs, 0.0), ph((size_t)p->npairs * 2 * PL * 2, 0.0);
  const long double wsig = 2.0L * kPi2 / N_sigma, P2 = (long double)P * P;
  for (int j = 0; j < p->npairs; ++j) {
    long double a = 0, sx = 1, sy = 0, scale = 0, c = 0;
    if (j < nreal) {
      const int ip = j / half, iq = j % half;
      const long double th = (iq + 0.5L) * wsig;
      a = kPi2 * rho[ip] / (2.0L * L);
      sx = cosl(th);
      sy = sinl(th);
      scale = 2.0L * wsig * 2.0L * b_c / P2;
      c = (long double)wr[ip] * powl((long double)rho[ip], 1.0L + gamma);
    }
    pd[4 * j] = (double)a;
    pd[4 * j + 1] = (double)sx;
    pd[4 * j + 2] = (double)sy;
    pd[4 * j + 3] = (double)scale;
    cp[j] = (double)c;
    const long double sd[2] = {sx, sy};
    for (int d = 0; d < 2; ++d)
      for (int n = -(N - 2); n <= N - 2; ++n) {
        const long double ang = a * sd[d] * n;
        const size_t o = (((size_t)j * 2 + d) * PL + (n + N - 2)) * 2;
        ph[o] = (double)cosl(ang);
        ph[o + 1] = (double)sinl(ang);
      }
  }
  p->S = std::max(1, std::min(p->npt, 1024));
  std::vector<double> twd(2 * P);
  for (int m = 0; m < P; ++m) {
    twd[2 * m] = (double)cosl(2 * kPi2 * m / P);
    twd[2 * m + 1] = (double)-sinl(2 * kPi2 * m / P);
  }
  std::vector<float> twf(twd.begin(), twd.end());
  std::vector<double> gj(gt);
  gj.insert(gj.end(), gw.begin(), gw.end());
  bzq_status s = BZQ_OK;
  double* d_pd = nullptr;
  double* d_gj = nullptr;
  DeviceArena tmp;
  if ((s = p->mem.get(&p->V, (size_t)p->npairs * p->nh * esz)) != BZQ_OK ||
      (s = p->mem.get(&p->ph, ph.size() * sizeof(double))) != BZQ_OK ||
      (s = p->mem.get(&p->cp, cp.size() * sizeof(double))) != BZQ_OK ||
      (s = p->mem.get(&p->tw, (size_t)P * 2 * esz)) != BZQ_OK ||
      (s = p->mem.get(&p->fc, (size_t)n1 * n1 * 2 * esz)) != BZQ_OK ||
      (s = p->mem.get(&p->fgrid, (size_t)P * P * esz)) != BZQ_OK ||
      (s = p->mem.get(&p->Qpart, (size_t)p->S * p->nh * 16)) != BZQ_OK ||
      (s = p->mem.get(&p->fin, (size_t)16 * p->nh * 16)) != BZQ_OK ||
      (s = p->mem.get(&p->q1, (size_t)N * N * 16)) != BZQ_OK ||
      (s = p->mem.get(&p->q2, (size_t)N * N * 16)) != BZQ_OK ||
      (s = p->mem.get(&p->fs, (size_t)N * N * 16)) != BZQ_OK ||
      (s = tmp.get(&d_pd, pd.size() * sizeof(double))) != BZQ_OK ||
      (s = tmp.get(&d_gj, gj.size() * sizeof(double))) != BZQ_OK) {
    delete p;
    return s;
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpyAsync(p->ph, ph.data(), ph.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(p->cp, cp.data(), cp.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_pd, pd.data(), pd.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_gj, gj.data(), gj.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = p->fp32 ? hipMemcpyAsync(p->tw, twf.data(), twf.size() * sizeof(float), hipMemcpyHostToDevice, st)
                : hipMemcpyAsync(p->tw, twd.data(), twd.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_table2d(p->V, d_pd, d_gj, n_jacobi, N, p->npairs, p->fp32, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete p;
    return fail(BZQ_EDEVICE, std::string("2-D plan creation: ") + hipGetErrorString(e));
  }
  *out = p;
  return BZQ_OK;
}

bzq_status bzq_collision2d(bzq_plan2d p, const double* f_hat, double* Q_hat, void* stream) {
  if (!p || !f_hat || !Q_hat) return fail(BZQ_EINVAL, "NULL argument");
  if (f_hat == Q_hat) return fail(BZQ_EINVAL, "f_hat and Q_hat must not overlap");
  hipError_t e = collide(p, f_hat, Q_hat, (hipStream_t)stream);
  if (e != hipSuccess) return fail(BZQ_EDEVICE, std::string("2-D collision: ") + hipGetErrorString(e));
  return BZQ_OK;
}

bzq_status bzq_step2d(bzq_plan2d p, double* f_hat, double dt, int n_steps, int method, void* stream) {
  if (!p || !f_hat) return fail(BZQ_EINVAL, "NULL argument");
  if (!(std::isfinite(dt) && dt > 0)) return fail(BZQ_EINVAL, "dt must be finite and > 0");
  if (n_steps < 0) return fail(BZQ_EINVAL, "n_steps must be >= 0");
  if (method != BZQ_HEUN && method != BZQ_RK4) return fail(BZQ_EINVAL, "unknown method");
  hipStream_t st = (hipStream_t)stream;
  const size_t n = (size_t)p->N * p->N;
  hipError_t e = hipSuccess;
  for (int i = 0; i < n_steps && e == hipSuccess; ++i) {
    if (method == BZQ_HEUN) {
      // q1 = Q(f), fs = f + dt q1, q2 = Q(fs), f += dt/2 (q1 + q2)
      if (e == hipSuccess) e = collide(p, f_hat, p->q1, st);
      if (e == hipSuccess) e = launch_axpy(p->fs, f_hat, dt, p->q1, n, st);
      if (e == hipSuccess) e = collide(p, p->fs, p->q2, st);
      if (e == hipSuccess) e = launch_heun(f_hat, p->q1, p->q2, 0.5 * dt, n, st);
    } else {
      // classical RK4; q1 = the stage's Q, q2 = the running sum, fs = the stage argument
      if (e == hipSuccess) e = collide(p, f_hat, p->q1, st);
      if (e == hipSuccess) e = launch_axpy(p->q2, f_hat, dt / 6.0, p->q1, n, st);
      if (e == hipSuccess) e = launch_axpy(p->fs, f_hat, 0.5 * dt, p->q1, n, st);
      if (e == hipSuccess) e = collide(p, p->fs, p->q1, st);
      if (e == hipSuccess) e = launch_axpy(p->q2, p->q2, dt / 3.0, p->q1, n, st);
      if (e == hipSuccess) e = launch_axpy(p->fs, f_hat, 0.5 * dt, p->q1, n, st);
      if (e == hipSuccess) e = collide(p, p->fs, p->q1, st);
      if (e == hipSuccess) e = launch_axpy(p->q2, p->q2, dt / 3.0, p->q1, n, st);
      if (e == hipSuccess) e = launch_axpy(p->fs, f_hat, dt, p->q1, n, st);
      if (e == hipSuccess) e = collide(p, p->fs, p->q1, st);
      if (e == hipSuccess) e = launch_axpy(f_hat, p->q2, dt / 6.0, p->q1, n, st);
    }
  }
  if (e != hipSuccess) return fail(BZQ_EDEVICE, std::string("2-D step: ") + hipGetErrorString(e));
  return BZQ_OK;
}

bzq_status bzq_plan2d_destroy(bzq_plan2d p) {
  if (!p) return BZQ_OK;
  (void)hipDeviceSynchronize();
  delete p;
  return BZQ_OK;
}

}  // extern "C"
