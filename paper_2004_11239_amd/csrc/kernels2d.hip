// Device kernels of the two-dimensional operator (d = 2) for gfx950.
//
// Same method as the 3-D path (Section 4, eq. realQ, with the circle in place
// of the sphere), but a whole padded P x P plane of one pair-two fits in LDS,
// so one workgroup carries a pair-two through every step with no intermediate
// in HBM: modulation of the compact spectrum by the separable phases of two
// antipodal pairs packed as E_A + i E_B, inverse FFT along axis 2 (the N-1 rows
// that hold modes) and axis 1, the product with f on the padded grid, forward
// FFT along axis 1 and axis 2 (kept rows only), separation of the two pairs by
// Hermitian symmetry, the real weight 2 w_sigma Re(e^{-ix} F)/P^2 times e^{ix}
// and c_p = w_rho rho^{1+gamma}, and FP64 accumulation in registers over the
// pair-twos s, s + S, ... of workgroup s.  A last kernel sums the S partial
// accumulators in a fixed order and completes the spectrum by Hermitian
// symmetry.  The FFTs are the LDS Stockham passes of fft.hpp; at N = 64 the
// same pipeline runs with the register passes of the 3-D plane kernel
// (k_collide2d_reg in kernels.hip).
//
// Layouts: compact spectra are centred, index i <-> k = i - (N/2 - 1); mode c =
// i2 (N-1) + i1 (i1 fastest), mirror nn - 1 - c; the half spectrum is c <=
// (nn - 1)/2.  In LDS the plane is buf[x (P+1) + y], x along axis 1.
#include "fft.hpp"
#include "kernels.hpp"
#include "kernels2d.hpp"

namespace bzq {
namespace {

__device__ __forceinline__ int posK2(int i, int h, int P) {
  const int k = i - (h - 1);
  return k >= 0 ? k : k + P;
}
struct RowsK {
  int ld, h, P;
  __device__ int operator()(int p) const { return posK2(p, h, P) * ld; }
};
struct Cols {
  __device__ int operator()(int p) const { return p; }
};

template <typename T>
__device__ __forceinline__ cx<T> cvt(double2 v) {
  return cx<T>{(T)v.x, (T)v.y};
}
__device__ __forceinline__ cx<double> d2(double2 v) { return cx<double>{v.x, v.y}; }

// (1 - cos Y) / Y^2, even in Y: power series below |Y| = 2
__device__ double c1m(double Y) {
  Y = fabs(Y);
  if (Y >= 2.0) return (1.0 - cos(Y)) / (Y * Y);
  const double z = Y * Y;
  double acc = 0.0, term = 0.5;   // 1/2! , then (-1)^k z^k / (2k+2)!
  for (int k = 0; k < 14; ++k) {
    acc += term;
    term *= -z / ((2.0 * k + 3.0) * (2.0 * k + 4.0));
  }
  return acc;
}

// Real weight of pair j at half-spectrum mode c:
//   V = 2 w_sigma Re(e^{-ix} F(k, rho, sigma)) / P^2,
//   Re(e^{-ix} F) = 2 c \int t^{-(s+1/2)} (1-t)^{-(r+1/2)}
//                   [ 2 sin(x(1-t)) sin(xt)/t cos Y - cos x 4 y^2 (1-t) c1m(Y) ] dt,
//   x = a k.sigma, y = a k.sigma_perp, Y = 2 y sqrt(t(1-t)).
// pd[j] = {a, sigma_x, sigma_y, 2 w_sigma 2 c / P^2}; gj = {t[nj], w[nj]}.
template <typename TV>
__global__ void k_table2d(TV* __restrict__ V, const double* __restrict__ pd, const double* __restrict__ gj,
                          int nj, int N, int npairs) {
  const int n1 = N - 1, h = N / 2, nh = (n1 * n1 + 1) / 2;
  const size_t total = (size_t)npairs * nh;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / nh), c = (int)(e - (size_t)j * nh);
    const double* q = pd + 4 * j;
    if (q[3] == 0.0) {
      V[e] = TV(0);
      continue;
    }
    const int i2 = c / n1, i1 = c - i2 * n1;
    const double k1 = i1 - h + 1, k2 = i2 - h + 1;
    const double x = q[0] * (k1 * q[1] + k2 * q[2]);
    const double y = q[0] * (-k1 * q[2] + k2 * q[1]);
    double acc = 0.0;
    const double cx0 = cos(x);
    for (int i = 0; i < nj; ++i) {
      const double t = gj[i], w = gj[nj + i];
      const double Y = 2.0 * y * sqrt(t * (1.0 - t));
      const double main = 2.0 * sin(x * (1.0 - t)) * sin(x * t) / t * cos(Y);
      const double loss = cx0 * 4.0 * y * y * (1.0 - t) * c1m(Y);
      acc += w * (main - loss);
    }
    V[e] = (TV)(q[3] * acc);
  }
}

// f on the padded grid, f(x) = sum_m f_m e^{2 pi i m.x / P}, one workgroup per
// grid column x2 = blockIdx.x: first R(k1) = sum_{k2} f_{k1 k2} e^{2 pi i k2 x2 / P}
// for the N-1 mode rows, then f(x1, x2) = sum_{k1} R(k1) e^{2 pi i k1 x1 / P} for
// all P rows: direct sums in FP64 (N (N + P) terms per column), rounded to T
// once.  Each sum is split over kPrepSplitR (first) or kPrepSplitX (second)
// threads, whose partial sums are added in a fixed order.  The workgroups
// also copy the compact spectrum fc (T precision).
constexpr int kPrepSplitR = 4, kPrepSplitX = 2;
template <typename T, int P, int NT>
__global__ __launch_bounds__(NT) void k_prep2d(const double2* __restrict__ f, cx<T>* __restrict__ fc,
                                               T* __restrict__ fgrid, int N) {
  constexpr int N1MAX = (2 * P) / 3 - 1;
  static_assert(NT >= kPrepSplitR * N1MAX && NT >= kPrepSplitX * P, "one partial sum per thread");
  __shared__ double2 tw[P];          // e^{+2 pi i m / P}
  __shared__ double2 part[kPrepSplitR][N1MAX];
  __shared__ double2 row[N1MAX];
  __shared__ double partx[kPrepSplitX][P];
  const int n1 = N - 1, h = N / 2, nn = n1 * n1;
  const int x2 = blockIdx.x;
  for (int i = threadIdx.x; i < P; i += NT) {
    double sn, cs;
    sincospi(2.0 * i / P, &sn, &cs);
    tw[i] = double2{cs, sn};
  }
  const int per = (nn + P - 1) / P;
  for (int c = x2 * per + threadIdx.x; c < min(nn, (x2 + 1) * per); c += NT) {
    const int i2 = c / n1, i1 = c - i2 * n1;
    const int a = (i1 - h + 1 + N) % N, b = (i2 - h + 1 + N) % N;
    fc[c] = cvt<T>(f[(size_t)a * N + b]);
  }
  __syncthreads();
  if (threadIdx.x < kPrepSplitR * n1) {
    const int q = threadIdx.x / n1, i1 = threadIdx.x - q * n1;
    const int a = (i1 - h + 1 + N) % N;
    double ax = 0.0, ay = 0.0;
    for (int i2 = q; i2 < n1; i2 += kPrepSplitR) {
      const int k2 = i2 - h + 1, b = (k2 + N) % N;
      int m = (k2 * x2) % P;
      if (m < 0) m += P;
      const double2 w = tw[m], v = f[(size_t)a * N + b];
      ax += v.x * w.x - v.y * w.y;
      ay += v.x * w.y + v.y * w.x;
    }
    part[q][i1] = double2{ax, ay};
  }
  __syncthreads();
  if (threadIdx.x < n1) {
    double2 t = part[0][threadIdx.x];
    for (int q = 1; q < kPrepSplitR; ++q) {
      t.x += part[q][threadIdx.x].x;
      t.y += part[q][threadIdx.x].y;
    }
    row[threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x < kPrepSplitX * P) {
    const int q = threadIdx.x / P, x1 = threadIdx.x - q * P;
    double acc = 0.0;
    for (int i1 = q; i1 < n1; i1 += kPrepSplitX) {
      const int k1 = i1 - h + 1;
      int m = (k1 * x1) % P;
      if (m < 0) m += P;
      const double2 w = tw[m];
      acc += row[i1].x * w.x - row[i1].y * w.y;    // Re(row e^{+i phi})
    }
    partx[q][x1] = acc;
  }
  __syncthreads();
  for (int x1 = threadIdx.x; x1 < P; x1 += NT) {
    double acc = partx[0][x1];
    for (int q = 1; q < kPrepSplitX; ++q) acc += partx[q][x1];
    fgrid[x1 * P + x2] = (T)acc;
  }
}

template <typename T, int P, int NT>
__global__ __launch_bounds__(NT) void k_collide2d(const cx<T>* __restrict__ fc, const T* __restrict__ fgrid,
                                                  const T* __restrict__ V, const double2* __restrict__ ph,
                                                  const double* __restrict__ cp, const cx<T>* __restrict__ twg,
                                                  double2* __restrict__ Qpart, int N, int npt, int S) {
  constexpr int LD = P + 1;
  constexpr int NMAX = (2 * P) / 3;
  constexpr int OPT = (((NMAX - 1) * (NMAX - 1) + 1) / 2 + NT - 1) / NT;
  __shared__ cx<T> buf[P * LD];
  __shared__ cx<T> tw[P];
  const int n1 = N - 1, h = N / 2, nn = n1 * n1, nh = (nn + 1) / 2, PL = 2 * N - 3;
  const int s = blockIdx.x;
  for (int i = threadIdx.x; i < P; i += NT) tw[i] = twg[i];
  double accx[OPT], accy[OPT];
#pragma unroll
  for (int b = 0; b < OPT; ++b) accx[b] = accy[b] = 0.0;
  for (int pt = s; pt < npt; pt += S) {
    const int jA = 2 * pt, jB = jA + 1;
    const double2* phA = ph + (size_t)jA * 2 * PL + (N - 2);
    const double2* phB = phA + 2 * PL;
    for (int i = threadIdx.x; i < P * LD; i += NT) buf[i] = cx<T>{0, 0};
    __syncthreads();
    // modulation: Z_m = f_m (E_A(m) + i E_B(m)), E(m) = e^{-i pi rho m.sigma / L}
    for (int c = threadIdx.x; c < nn; c += NT) {
      const int i2 = c / n1, i1 = c - i2 * n1;
      const int k1 = i1 - h + 1, k2 = i2 - h + 1;
      const cx<double> eA = cmul(d2(phA[-2 * k1]), d2(phA[PL - 2 * k2]));
      const cx<double> eB = cmul(d2(phB[-2 * k1]), d2(phB[PL - 2 * k2]));
      const cx<T> m = {(T)(eA.x - eB.y), (T)(eA.y + eB.x)};
      buf[posK2(i1, h, P) * LD + posK2(i2, h, P)] = cmul(fc[c], m);
    }
    __syncthreads();
    fft_pencils<T, P, +1, NT, P>(buf, n1, RowsK{LD, h, P}, 1, tw);
    fft_pencils<T, P, +1, NT, P>(buf, P, Cols{}, LD, tw);
    for (int e = threadIdx.x; e < P * P; e += NT) {
      const int x = e / P, y = e - x * P;
      buf[x * LD + y] = cscale(buf[x * LD + y], fgrid[e]);
    }
    __syncthreads();
    fft_pencils<T, P, -1, NT, P>(buf, P, Cols{}, LD, tw);
    fft_pencils<T, P, -1, NT, P>(buf, n1, RowsK{LD, h, P}, 1, tw);
    const double cA = cp[jA], cB = cp[jB];
#pragma unroll
    for (int b = 0; b < OPT; ++b) {
      const int c = threadIdx.x + b * NT;
      if (c < nh) {
        const int i2 = c / n1, i1 = c - i2 * n1;
        const int k1 = i1 - h + 1, k2 = i2 - h + 1;
        const cx<T> w1 = buf[posK2(i1, h, P) * LD + posK2(i2, h, P)];
        const cx<T> w2 = buf[posK2(n1 - 1 - i1, h, P) * LD + posK2(n1 - 1 - i2, h, P)];
        // h_A = (w(k) + conj w(-k))/2,  h_B = (w(k) - conj w(-k))/(2i)
        const cx<double> hA = {0.5 * ((double)w1.x + (double)w2.x), 0.5 * ((double)w1.y - (double)w2.y)};
        const cx<double> hB = {0.5 * ((double)w1.y + (double)w2.y), -0.5 * ((double)w1.x - (double)w2.x)};
        const double vA = cA * (double)V[(size_t)jA * nh + c];
        const double vB = cB * (double)V[(size_t)jB * nh + c];
        const cx<double> eA = cmul(d2(phA[k1]), d2(phA[PL + k2]));
        const cx<double> eB = cmul(d2(phB[k1]), d2(phB[PL + k2]));
        const cx<double> tA = cmul(eA, hA), tB = cmul(eB, hB);
        accx[b] += vA * tA.x + vB * tB.x;
        accy[b] += vA * tA.y + vB * tB.y;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < OPT; ++b) {
    const int c = threadIdx.x + b * NT;
    if (c < nh) Qpart[(size_t)s * nh + c] = double2{accx[b], accy[b]};
  }
}

// Sum of the S partial accumulators in two fixed-order stages.  Stage one:
// workgroup (bx, g) sums, for the 64 half-spectrum modes c = 64 bx + lane, the
// partials s of chunk g (its 4 waves take every 4th s, then add in wave order)
// into tmp[g][c].  Stage two: Q (N^2, FFT order) = sum over g < G of tmp[g],
// Hermitian completion, Nyquist rows and columns 0.
constexpr int kFinChunks = 16;

__global__ __launch_bounds__(256) void k_finpart2d(const double2* __restrict__ Qpart, double2* __restrict__ tmp,
                                                   int nh, int S) {
  __shared__ double2 red[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane, g = blockIdx.y;
  const int per = (S + kFinChunks - 1) / kFinChunks;
  const int s0 = g * per, s1 = min(S, s0 + per);
  double sx = 0.0, sy = 0.0;
  if (c < nh) {
    for (int s = s0 + wv; s < s1; s += 4) {
      const double2 v = Qpart[(size_t)s * nh + c];
      sx += v.x;
      sy += v.y;
    }
  }
  red[wv][lane] = double2{sx, sy};
  __syncthreads();
  if (wv == 0 && c < nh) {
    double2 t = red[0][lane];
    for (int w = 1; w < 4; ++w) {
      t.x += red[w][lane].x;
      t.y += red[w][lane].y;
    }
    tmp[(size_t)g * nh + c] = t;
  }
}

__global__ void k_finalize2d(const double2* __restrict__ tmp, double2* __restrict__ Q, int N) {
  const int n1 = N - 1, h = N / 2, nn = n1 * n1, nh = (nn + 1) / 2, cmid = (nn - 1) / 2;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N * N; e += gridDim.x * blockDim.x) {
    const int a = e / N, b = e - a * N;
    if (a == h || b == h) {
      Q[e] = double2{0.0, 0.0};
      continue;
    }
    const int k1 = a < h ? a : a - N, k2 = b < h ? b : b - N;
    const int c = (k2 + h - 1) * n1 + (k1 + h - 1);
    const bool mirror = c > cmid;
    const int cc = mirror ? nn - 1 - c : c;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int g = 0; g < kFinChunks; ++g) {
      const double2 v = tmp[(size_t)g * nh + cc];
      sx += v.x;
      sy += v.y;
    }
    Q[e] = double2{sx, mirror ? -sy : sy};
  }
}

inline int grid2(size_t n) {
  size_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : g > 4096 ? 4096 : g);
}

// Threads of the pipeline workgroup: the kernel waits on LDS and barriers, so
// as many waves as the registers allow (FP32: 16 waves, about 100 VGPRs; FP64:
// 8 waves, about 230 VGPRs, no spills).  Measured at N = 32 and 64: 1.1-1.3x
// faster than 4 waves.
template <typename T, int P>
constexpr int collideThreads() {
  return sizeof(T) == 4 ? 1024 : 512;
}

template <typename T, int P>
hipError_t collide2d_t(const double* f_hat, void* fc, void* fgrid, const void* V, const double* ph,
                       const double* cp, const void* tw, double* Qpart, int N, int npt, int S, hipStream_t st) {
  constexpr int NT = collideThreads<T, P>();
  hipLaunchKernelGGL((k_prep2d<T, P, 256>), dim3(P), dim3(256), 0, st, (const double2*)f_hat, (cx<T>*)fc,
                     (T*)fgrid, N);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // N = 64 with one pair-two per workgroup: the register-FFT pipeline (kernels.hip)
  if constexpr (P == 96)
    if (N == 64 && S >= npt) return launch_collide2d_reg(fc, fgrid, V, ph, cp, Qpart, N, npt, S, sizeof(T) == 4, st);
  hipLaunchKernelGGL((k_collide2d<T, P, NT>), dim3(S), dim3(NT), 0, st, (const cx<T>*)fc, (const T*)fgrid,
                     (const T*)V, (const double2*)ph, cp, (const cx<T>*)tw, (double2*)Qpart, N, npt, S);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_table2d(void* V, const double* pd, const double* gj, int nj, int N, int npairs, bool fp32,
                          hipStream_t st) {
  const size_t n = (size_t)npairs * (((N - 1) * (N - 1) + 1) / 2);
  if (fp32)
    hipLaunchKernelGGL(k_table2d<float>, dim3(grid2(n)), dim3(256), 0, st, (float*)V, pd, gj, nj, N, npairs);
  else
    hipLaunchKernelGGL(k_table2d<double>, dim3(grid2(n)), dim3(256), 0, st, (double*)V, pd, gj, nj, N, npairs);
  return hipGetLastError();
}

hipError_t launch_collision2d(const double* f_hat, double* Q_hat, void* fc, void* fgrid, const void* V,
                              const double* ph, const double* cp, const void* tw, double* Qpart, double* tmp, int N,
                              int P, int npt, int S, bool fp32, hipStream_t st) {
  hipError_t e = hipSuccess;
#define CASE(PP)                                                                                       \
  case PP:                                                                                             \
    e = fp32 ? collide2d_t<float, PP>(f_hat, fc, fgrid, V, ph, cp, tw, Qpart, N, npt, S, st)          \
             : collide2d_t<double, PP>(f_hat, fc, fgrid, V, ph, cp, tw, Qpart, N, npt, S, st);        \
    break;
  switch (P) {
    CASE(12) CASE(24) CASE(36) CASE(48) CASE(72) CASE(96)
    default: return hipErrorInvalidValue;
  }
#undef CASE
  if (e != hipSuccess) return e;
  const int nh = ((N - 1) * (N - 1) + 1) / 2;
  hipLaunchKernelGGL(k_finpart2d, dim3((nh + 63) / 64, kFinChunks), dim3(256), 0, st, (const double2*)Qpart,
                     (double2*)tmp, nh, S);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_finalize2d, dim3(grid2((size_t)N * N)), dim3(256), 0, st, (const double2*)tmp,
                     (double2*)Q_hat, N);
  return hipGetLastError();
}

}  // namespace bzq
