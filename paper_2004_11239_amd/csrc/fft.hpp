// Device-side FFT building blocks for gfx950: complex arithmetic, small
// in-register DFTs (radix 2, 3, 4, 6, 8, 12) and Stockham autosort passes over
// pencils resident in LDS.
//
// The convolutions of the fast method (Section 4, eq. realQ) are evaluated by
// zero-padded 3-D FFTs of size P = 3N/2 per axis; P and the unpadded N are of
// the form 2^a 3^b, so every length here factors into the radices below:
//   8 = 8, 12 = 12, 16 = 4*4, 24 = 4*6, 32 = 4*8, 36 = 6*6, 48 = 4*12,
//   64 = 8*8, 72 = 6*12, 96 = 8*12.
// Convention: X[q] = sum_r x[r] e^{SIGN 2 pi i r q / n}, unnormalised.
#pragma once
#include <hip/hip_runtime.h>

namespace bzq {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// i * SIGN * a
template <int SIGN, typename T>
__host__ __device__ __forceinline__ cx<T> rot(cx<T> a) {
  return SIGN > 0 ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

// ---------------------------------------------------------------- small DFTs
template <int SIGN, typename T>
__host__ __device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int SIGN, typename T>
__host__ __device__ __forceinline__ void dft3(cx<T>& a, cx<T>& b, cx<T>& c) {
  const T s3 = T(0.86602540378443864676372317075294);
  cx<T> t1 = cadd(b, c);
  cx<T> t2 = {a.x - T(0.5) * t1.x, a.y - T(0.5) * t1.y};
  cx<T> d = csub(b, c);
  cx<T> t3 = rot<SIGN>(cx<T>{s3 * d.x, s3 * d.y});
  a = cadd(a, t1);
  b = cadd(t2, t3);
  c = csub(t2, t3);
}

template <int SIGN, typename T>
__host__ __device__ __forceinline__ void dft4(cx<T>& a, cx<T>& b, cx<T>& c, cx<T>& d) {
  cx<T> s0 = cadd(a, c), d0 = csub(a, c);
  cx<T> s1 = cadd(b, d), d1 = rot<SIGN>(csub(b, d));
  a = cadd(s0, s1);
  c = csub(s0, s1);
  b = cadd(d0, d1);
  d = csub(d0, d1);
}

// radix-2 decimation in time over two DFT4s
template <int SIGN, typename T>
__host__ __device__ __forceinline__ void dft8(cx<T>* v) {
  const T h = T(0.70710678118654752440084436210485);
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<SIGN>(e0, e1, e2, e3);
  dft4<SIGN>(o0, o1, o2, o3);
  // o_q *= e^{SIGN 2 pi i q / 8}
  o1 = cx<T>{h * (o1.x - T(SIGN) * o1.y), h * (o1.y + T(SIGN) * o1.x)};
  o2 = rot<SIGN>(o2);
  o3 = cx<T>{h * (-o3.x - T(SIGN) * o3.y), h * (-o3.y + T(SIGN) * o3.x)};
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// Good-Thomas: 6 = 2 x 3, input n = (3 n1 + 2 n2) mod 6, output k = (3 k1 + 4 k2) mod 6
template <int SIGN, typename T>
__host__ __device__ __forceinline__ void dft6(cx<T>* v) {
  cx<T> a0 = v[0], a1 = v[2], a2 = v[4];   // n1 = 0: n2 = 0,1,2 -> n = 0,2,4
  cx<T> b0 = v[3], b1 = v[5], b2 = v[1];   // n1 = 1: n = 3,5,1
  dft2<SIGN>(a0, b0);
  dft2<SIGN>(a1, b1);
  dft2<SIGN>(a2, b2);
  dft3<SIGN>(a0, a1, a2);                  // k1 = 0
  dft3<SIGN>(b0, b1, b2);                  // k1 = 1
  v[0] = a0; v[4] = a1; v[2] = a2;         // k = 4 k2 mod 6
  v[3] = b0; v[1] = b1; v[5] = b2;         // k = 3 + 4 k2 mod 6
}

// Good-Thomas: 12 = 4 x 3, input n = (3 n1 + 4 n2) mod 12, output k = (9 k1 + 4 k2) mod 12
template <int SIGN, typename T>
__host__ __device__ __forceinline__ void dft12(cx<T>* v) {
  cx<T> u[4][3];
#pragma unroll
  for (int n2 = 0; n2 < 3; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) u[n1][n2] = v[(3 * n1 + 4 * n2) % 12];
    dft4<SIGN>(u[0][n2], u[1][n2], u[2][n2], u[3][n2]);
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    dft3<SIGN>(u[k1][0], u[k1][1], u[k1][2]);
#pragma unroll
    for (int k2 = 0; k2 < 3; ++k2) v[(9 * k1 + 4 * k2) % 12] = u[k1][k2];
  }
}

template <int R, int SIGN, typename T>
__host__ __device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 2) {
    dft2<SIGN>(v[0], v[1]);
  } else if constexpr (R == 3) {
    dft3<SIGN>(v[0], v[1], v[2]);
  } else if constexpr (R == 4) {
    dft4<SIGN>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 6) {
    dft6<SIGN>(v);
  } else if constexpr (R == 8) {
    dft8<SIGN>(v);
  } else if constexpr (R == 12) {
    dft12<SIGN>(v);
  } else {
    static_assert(R == 2, "unsupported radix");
  }
}

// ------------------------------------------------------------- radix plans
template <int P>
struct RadixPlan;
template <> struct RadixPlan<8>  { static constexpr int R0 = 8, R1 = 1, R2 = 1; };
template <> struct RadixPlan<12> { static constexpr int R0 = 12, R1 = 1, R2 = 1; };
template <> struct RadixPlan<16> { static constexpr int R0 = 4, R1 = 4, R2 = 1; };
template <> struct RadixPlan<24> { static constexpr int R0 = 4, R1 = 6, R2 = 1; };
template <> struct RadixPlan<32> { static constexpr int R0 = 4, R1 = 8, R2 = 1; };
template <> struct RadixPlan<36> { static constexpr int R0 = 6, R1 = 6, R2 = 1; };
template <> struct RadixPlan<48> { static constexpr int R0 = 4, R1 = 12, R2 = 1; };
template <> struct RadixPlan<64> { static constexpr int R0 = 8, R1 = 8, R2 = 1; };
template <> struct RadixPlan<72> { static constexpr int R0 = 6, R1 = 12, R2 = 1; };
template <> struct RadixPlan<96> { static constexpr int R0 = 8, R1 = 12, R2 = 1; };
// three passes (LDS kernels only: these pencils do not fit the register file)
template <> struct RadixPlan<128> { static constexpr int R0 = 8, R1 = 4, R2 = 4; };
template <> struct RadixPlan<192> { static constexpr int R0 = 8, R1 = 4, R2 = 6; };

// ------------------------------------------------------ Stockham LDS passes
// One radix-R pass over `npencils` pencils of length P stored in LDS.
// Element e of pencil p lives at buf[addr(p) + e * es].  Butterfly j of a
// pencil reads elements j + r P/R (r < R), multiplies element r by
// w^{r (j mod NS)} with w = e^{SIGN 2 pi i / (NS R)}, applies the R-point DFT
// and writes element r to (j / NS) NS R + (j mod NS) + r NS.  Passes with
// NS = 1, R0, R0 R1 ... give the DFT in natural order (Stockham autosort).
// The caller must have synchronised before the call; the pass ends with a
// barrier.  `tw` holds e^{-2 pi i m / P}, m < P (LDS).
template <typename T, int P, int R, int NS, int SIGN, int BMAX, int NT, typename Addr>
__device__ __forceinline__ void stockham_pass(cx<T>* __restrict__ buf, int npencils, Addr addr,
                                              int es, const cx<T>* __restrict__ tw) {
  constexpr int NB = P / R;
  const int total = npencils * NB;
  cx<T> v[BMAX][R];
  int dst[BMAX];
#pragma unroll
  for (int b = 0; b < BMAX; ++b) {
    const int idx = threadIdx.x + b * NT;
    if (idx < total) {
      const int p = idx / NB;
      const int j = idx - p * NB;
      const int base = addr(p);
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[base + (j + r * NB) * es];
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[r * k * (P / (NS * R))];
          if constexpr (SIGN > 0) w.y = -w.y;
          v[b][r] = cmul(v[b][r], w);
        }
      }
      dft<R, SIGN>(v[b]);
      dst[b] = base + ((j / NS) * NS * R + (j % NS)) * es;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BMAX; ++b) {
    const int idx = threadIdx.x + b * NT;
    if (idx < total) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[b] + r * NS * es] = v[b][r];
    }
  }
  __syncthreads();
}

template <int MAXP, int P, int R, int NT>
struct Bmax {
  static constexpr int value = (MAXP * (P / R) + NT - 1) / NT;
};

// Full length-P transform of up to MAXP pencils (all passes).
template <typename T, int P, int SIGN, int NT, int MAXP, typename Addr>
__device__ __forceinline__ void fft_pencils(cx<T>* __restrict__ buf, int npencils, Addr addr, int es,
                                            const cx<T>* __restrict__ tw) {
  constexpr int R0 = RadixPlan<P>::R0;
  constexpr int R1 = RadixPlan<P>::R1;
  constexpr int R2 = RadixPlan<P>::R2;
  static_assert(R0 * R1 * R2 == P, "radix plan");
  stockham_pass<T, P, R0, 1, SIGN, Bmax<MAXP, P, R0, NT>::value, NT>(buf, npencils, addr, es, tw);
  if constexpr (R1 > 1)
    stockham_pass<T, P, R1, R0, SIGN, Bmax<MAXP, P, R1, NT>::value, NT>(buf, npencils, addr, es, tw);
  if constexpr (R2 > 1)
    stockham_pass<T, P, R2, R0 * R1, SIGN, Bmax<MAXP, P, R2, NT>::value, NT>(buf, npencils, addr, es, tw);
}

// ------------------------------------------------- compile-time twiddles
// cos and sin of 2 pi m / P in double precision, evaluated at compile time:
// quadrant reduction in exact integer arithmetic, then Taylor series on
// [0, pi/4] (the first dropped term is below 1e-20).
struct CosSin {
  double c, s;
};
constexpr double kPiD = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
constexpr CosSin cos_sin_2pi(int m, int P) {
  m %= P;
  if (m < 0) m += P;
  const int q = (4 * m) / P;          // quadrant
  const int rem = 4 * m - q * P;      // angle within quadrant = (pi/2) rem / P
  double c0 = 0.0, s0 = 0.0;
  if (2 * rem <= P) {                 // <= pi/4
    const double phi = 0.5 * kPiD * rem / P;
    c0 = taylor_cos(phi);
    s0 = taylor_sin(phi);
  } else {                            // use the complement pi/2 - phi
    const double psi = 0.5 * kPiD * (P - rem) / P;
    c0 = taylor_sin(psi);
    s0 = taylor_cos(psi);
  }
  switch (q & 3) {
    case 0: return {c0, s0};
    case 1: return {-s0, c0};
    case 2: return {-c0, -s0};
    default: return {s0, -c0};
  }
}

template <int P>
struct TwiddleTable {
  double c[P], s[P];
  constexpr TwiddleTable() : c{}, s{} {
    for (int m = 0; m < P; ++m) {
      const CosSin v = cos_sin_2pi(m, P);
      c[m] = v.c;
      s[m] = v.s;
    }
  }
};

// x * e^{SIGN 2 pi i m / P} with m known after unrolling; exact for m in {0, P/4, P/2, 3P/4}
template <int P, int SIGN, typename T>
__host__ __device__ __forceinline__ cx<T> twiddle_mul(cx<T> x, int m) {
  constexpr TwiddleTable<P> tw{};
  m %= P;
  if (m == 0) return x;
  if (4 * m == P) return rot<SIGN>(x);
  if (2 * m == P) return cx<T>{-x.x, -x.y};
  if (4 * m == 3 * P) return rot<-SIGN>(x);
  const T c = (T)tw.c[m];
  const T s = (T)(SIGN > 0 ? tw.s[m] : -tw.s[m]);
  return cx<T>{x.x * c - x.y * s, x.x * s + x.y * c};
}

// Length-P DFT of x[0..P) held in registers (all indices compile-time after
// unrolling), natural order in and out.  Four-step with P = R0 R1:
//   n = R1 n0 + n1, k = k0 + R0 k1;
//   Y[n1][k0] = w_P^{n1 k0} DFT_R0(x[R1 n0 + n1])[k0];  X[k0 + R0 k1] = DFT_R1(Y[.][k0])[k1].
// Zero inputs that are compile-time constants fold away (with -fno-signed-zeros).
template <int P, int SIGN, typename T>
__host__ __device__ __forceinline__ void fft_reg(cx<T>* x) {
  constexpr int R0 = RadixPlan<P>::R0;
  constexpr int R1 = RadixPlan<P>::R1;
  static_assert(RadixPlan<P>::R2 == 1, "register transforms take two-factor lengths");
  if constexpr (R1 == 1) {
    dft<R0, SIGN>(x);
  } else {
    cx<T> y[P];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
      cx<T> t[R0];
#pragma unroll
      for (int n0 = 0; n0 < R0; ++n0) t[n0] = x[R1 * n0 + n1];
      dft<R0, SIGN>(t);
#pragma unroll
      for (int k0 = 0; k0 < R0; ++k0) y[n1 * R0 + k0] = twiddle_mul<P, SIGN>(t[k0], n1 * k0);
    }
#pragma unroll
    for (int k0 = 0; k0 < R0; ++k0) {
      cx<T> t[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) t[n1] = y[n1 * R0 + k0];
      dft<R1, SIGN>(t);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) x[k0 + R0 * k1] = t[k1];
    }
  }
}

// Half of a length-P transform, P = 2Q, by one decimation-in-frequency step:
// with u[n] = (x[n] + (-1)^PAR x[n+Q]) w_P^{PAR n}, n < Q, the outputs of
// parity PAR are X[2j + PAR] = DFT_Q(u)[j].  `get(n)` returns input n (n is a
// compile-time constant after unrolling, so structurally zero inputs fold
// away).  On return u[j] = X[2j + PAR].  With GROUP > 0 the inputs are
// fetched GROUP pairs at a time (a scheduling barrier after each group), which
// bounds the registers held by loads in flight.
template <int P, int SIGN, int PAR, int GROUP = 0, typename T, typename Get>
__host__ __device__ __forceinline__ void dft_half_dif(Get get, cx<T>* u) {
  constexpr int Q = P / 2;
#pragma unroll
  for (int n = 0; n < Q; ++n) {
    const cx<T> a = get(n), b = get(n + Q);
    if constexpr (PAR == 0) {
      u[n] = cadd(a, b);
    } else {
      u[n] = twiddle_mul<P, SIGN>(csub(a, b), n);
    }
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (GROUP > 0)
      if ((n + 1) % GROUP == 0) __builtin_amdgcn_sched_barrier(0);
#endif
  }
  fft_reg<Q, SIGN>(u);
}

// A quarter of a length-P transform, P = 4 Q4, by one radix-4 decimation step
// in frequency: with u[n] = w_P^{R n} sum_{a < 4} i^{SIGN a R} x[n + a Q4],
// n < Q4, the outputs of class R are X[4j + R] = DFT_Q4(u)[j].  `get(n)` as
// for dft_half_dif.  On return u[j] = X[4j + R].
template <int P, int SIGN, int R, typename T, typename Get>
__host__ __device__ __forceinline__ void dft_quarter_dif(Get get, cx<T>* u) {
  constexpr int Q4 = P / 4;
  static_assert(P % 4 == 0 && R >= 0 && R < 4, "quarter split needs P = 4 Q4 and R < 4");
#pragma unroll
  for (int n = 0; n < Q4; ++n) {
    const cx<T> x0 = get(n), x1 = get(n + Q4), x2 = get(n + 2 * Q4), x3 = get(n + 3 * Q4);
    cx<T> v;
    if constexpr (R == 0) {
      v = cadd(cadd(x0, x2), cadd(x1, x3));
    } else if constexpr (R == 2) {
      v = csub(cadd(x0, x2), cadd(x1, x3));
    } else if constexpr (R == 1) {
      v = cadd(csub(x0, x2), rot<SIGN>(csub(x1, x3)));      // i^{SIGN a}: 1, i^SIGN, -1, -i^SIGN
    } else {
      v = cadd(csub(x0, x2), rot<-SIGN>(csub(x1, x3)));     // i^{3 SIGN a}: 1, i^-SIGN, -1, -i^-SIGN
    }
    u[n] = twiddle_mul<P, SIGN>(v, n * R);
  }
  fft_reg<Q4, SIGN>(u);
}

}  // namespace bzq
