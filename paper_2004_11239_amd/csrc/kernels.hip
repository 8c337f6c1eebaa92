// Device kernels of the fast collision operator (Section 4, eq. realQ) for gfx950.
//
// One evaluation Q = Q(f, f) runs, per chunk of quadrature pairs:
//   zinv : modulation by the separable phases e^{-i pi rho m.sigma / L} of two
//          antipodal pairs packed as one complex spectrum Z = f (E_A + i E_B),
//          zero padding to P = 3N/2, inverse FFT along axis 3;
//   plane: per (pair-two, z) plane in LDS, inverse FFT along axes 2 and 1, the
//          pointwise product with f(v) on the padded grid, forward FFT along
//          axes 1 and 2 (only the N-1 kept modes leave the kernel);
//   zfwd : forward FFT along axis 3, separation of the two packed pairs by
//          Hermitian symmetry, the weight 2 w_sigma Re(e^{-ix} F) e^{ix} c_p and
//          the FP64 accumulation over pairs.
// Layouts: compact spectra are centred, index i <-> k = i - (N/2 - 1),
// i < N-1; c = i2 (N-1) + i1 indexes a pencil along axis 3 (i1 fastest, so
// that one thread per pencil reads and writes coalesced).  The mirror of
// pencil c is (N-1)^2 - 1 - c and the mirror of i3 is N-2-i3.  The compact
// copy of f is fc[i3][c]; the first intermediate is A[pt][z][c].  The second,
// B[pt][z][slot], is folded so that a pencil and its mirror sit at the same
// offset of two aligned halves: slot(c) = c for c <= cmid and
// nhp + (nn - 1 - c) otherwise, nhp = nh rounded up to 16 (the centre pencil
// cmid is stored in both halves).
//
// Two implementations of each FFT stage exist: a register one (one thread
// holds a whole length-P pencil, twiddles are compile-time constants and the
// zero padding folds away) used wherever a pencil fits the register file, and
// an LDS Stockham one used otherwise (FP64 at P >= 72) and by the last stage.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "fft.hpp"
#include "funk_hecke.hpp"
#include "kernels.hpp"

namespace bzq {

namespace {

// Tiles of the LDS z kernels (measured at 128^3, P = 192: 16 z-inverse pencils
// per workgroup, 5.4 / 11.3 ms FP32 / FP64 against 7.3 / 16.8 with 32; 8
// z-forward pencils, 7.3 ms FP32 against 14.8 with 16)
constexpr int K1_TP = 16;   // pencils per zinv workgroup
constexpr int K3_TQ = 8;    // half-spectrum pencils per zfwd workgroup
constexpr int NT_SMALL = 256;

template <int P>
struct PlaneThreads {
  static constexpr int value = P >= 72 ? 512 : 256;
};

// half-spectrum pencil count rounded up to the zfwd tile, and the folded B slot
__host__ __device__ __forceinline__ int nh_pad(int N) {
  const int nh = ((N - 1) * (N - 1) + 1) / 2;
  return (nh + 15) / 16 * 16;
}
__device__ __forceinline__ int fold_slot(int c, int nn, int nhp) {
  const int cmid = (nn - 1) / 2;
  return c <= cmid ? c : nhp + (nn - 1 - c);
}

// position of centred index i (k = i - (h-1)) in a length-P FFT-order axis
__device__ __forceinline__ int posK(int i, int h, int P) {
  const int k = i - (h - 1);
  return k >= 0 ? k : k + P;
}

// Largest N - 1 that a length-P axis carries: P - 1 on an unpadded grid
// (P = N), 2P/3 - 1 on a padded one (P = 3N/2).
template <int P>
constexpr int maxN1() {
  return (P == 8 || P == 16 || P == 24 || P == 32 || P == 48 || P == 64 || P == 128) ? P - 1 : 2 * P / 3 - 1;
}

// n element copies (element e: v = load(e), then store(e, v)) by NT threads,
// every load of a thread issued before its first store, so that its loads are
// in flight together rather than one memory round trip per element.  MAXN
// bounds n at compile time.
template <typename V, int MAXN, int NT, typename Load, typename Store>
__device__ __forceinline__ void staged_copy(int n, Load load, Store store) {
  constexpr int K = (MAXN + NT - 1) / NT;
  V v[K];
#pragma unroll
  for (int b = 0; b < K; ++b) {
    const int e = (int)threadIdx.x + b * NT;
    if (e < n) v[b] = load(e);
  }
#pragma unroll
  for (int b = 0; b < K; ++b) {
    const int e = (int)threadIdx.x + b * NT;
    if (e < n) store(e, v[b]);
  }
}

// Workgroup barrier that orders LDS accesses only: global loads issued before
// it stay in flight (used where weights for the next step are prefetched).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Non-temporal access for the plane stage, which streams the first
// intermediate in and the second out (each element is touched once there);
// measured faster than ordinary accesses for that stage, while the z stages
// are faster with ordinary ones.
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ cx<T> ld_nt(const cx<T>* p) {
  const vec2<T> v = __builtin_nontemporal_load(reinterpret_cast<const vec2<T>*>(p));
  return cx<T>{v.x, v.y};
}
// A row input of the plane's four-way row passes, which four waves of a
// workgroup read: non-temporal in FP32 (measured faster at P = 96), ordinary
// in FP64, where streaming it made every wave fetch it again (64^3 plane
// 35.4 -> 32.3 ms with ordinary loads in the four-wave kernel).
template <typename T>
__device__ __forceinline__ cx<T> ld_row(const cx<T>* p) {
  if constexpr (sizeof(T) == 8) return *p;
  else return ld_nt(p);
}
template <typename T>
__device__ __forceinline__ void st_nt(cx<T>* p, cx<T> v) {
  __builtin_nontemporal_store(vec2<T>{v.x, v.y}, reinterpret_cast<vec2<T>*>(p));
}
template <typename T>
__device__ __forceinline__ cx<T> to_cx(double2 v) {
  return {(T)v.x, (T)v.y};
}
__device__ __forceinline__ cx<double> d2c(double2 v) { return {v.x, v.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cvt(cx<double> v) {
  return {(T)v.x, (T)v.y};
}
// Element i of an array whose base is the same for the whole wave, addressed
// by a 32-bit offset: the access takes the scalar-base plus vector-offset form,
// so unrolled loops over strided elements do not hold one 64-bit address
// constant per element in scalar registers.  The byte offset must be < 2^32.
template <typename U>
__device__ __forceinline__ U* at32(U* base, unsigned i) {
  return reinterpret_cast<U*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(U));
}
template <typename U>
__device__ __forceinline__ const U* at32(const U* base, unsigned i) {
  return reinterpret_cast<const U*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(U));
}

struct RowAddr {
  int ld;
  __device__ int operator()(int p) const { return p * ld; }
};
struct RowKAddr {
  int ld, h, P;
  __device__ int operator()(int p) const { return posK(p, h, P) * ld; }
};
struct ColAddr {
  __device__ int operator()(int p) const { return p; }
};

// Adds a thread's FP64 sums acc[b] into Qpart[idx(b)] (idx < 0: none), or
// writes them when `first`.  Every old value is read before any is written
// (in one read-add-write loop each read would wait for the write before it,
// since the compiler cannot tell that the elements differ), and the sums are
// formed outside the guarded stores, so that no store waits for the one
// before it.
template <int OPT, typename Idx>
__device__ __forceinline__ void add_partials(double2* __restrict__ Qpart, const double* accx,
                                             const double* accy, bool first, Idx idx) {
  long long qi[OPT];
  double2 v[OPT];
#pragma unroll
  for (int b = 0; b < OPT; ++b) {
    qi[b] = idx(b);
    v[b] = double2{0.0, 0.0};
  }
  if (!first) {
#pragma unroll
    for (int b = 0; b < OPT; ++b)
      if (qi[b] >= 0) v[b] = Qpart[qi[b]];
  }
#pragma unroll
  for (int b = 0; b < OPT; ++b) {
    v[b] = double2{v[b].x + accx[b], v[b].y + accy[b]};
    // an empty statement that uses the sums keeps them from being moved into
    // the guarded stores (where each would wait for the store before it)
    asm volatile("" ::"v"(v[b].x), "v"(v[b].y));
  }
#pragma unroll
  for (int b = 0; b < OPT; ++b)
    if (qi[b] >= 0) Qpart[qi[b]] = v[b];
}

// ------------------------------------------------------------------ ingest
// With flag != nullptr, flag[0] is set to 1 when any value read (every entry
// off the Nyquist planes) is NaN or Inf: the input check of the a0 stage.
template <typename T>
__global__ void k_ingest(PtrPack fin, cx<T>* __restrict__ fc, size_t fc_stride, int N, int* __restrict__ flag) {
  const int n1 = N - 1, h = N / 2;
  const int total = n1 * n1 * n1;
  const double2* __restrict__ f = (const double2*)fin.p[blockIdx.y];
  fc += blockIdx.y * fc_stride;
  bool bad = false;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int i3 = e / (n1 * n1);
    const int i2 = (e / n1) % n1;
    const int i1 = e % n1;
    const int a = (i1 - h + 1 + N) % N, b = (i2 - h + 1 + N) % N, c = (i3 - h + 1 + N) % N;
    const double2 v = f[((size_t)a * N + b) * N + c];
    bad |= !isfinite(v.x) || !isfinite(v.y);
    fc[e] = to_cx<T>(v);
  }
  if (bad && flag) flag[0] = 1;
}

// -------------------------------------------------------------------- zinv
// LDS kernel for pencils that do not fit the register file: K1_TP pencils
// per workgroup.  The pair-two's phase factors are staged in LDS once per
// workgroup (axes 1 and 2 per pencil, axis 3 per height) and multiplied in
// the order of the register kernels' modulation.
template <typename T, int P, int NT>
__global__ __launch_bounds__(NT) void k_zinv(const cx<T>* __restrict__ fc, const double2* __restrict__ ph,
                                             cx<T>* __restrict__ A, const cx<T>* __restrict__ twg, int N,
                                             int pair0, int mode, CellStrides cs) {
  constexpr int LD = P + 1, MN1 = maxN1<P>();
  fc += blockIdx.z * cs.fc;
  A += blockIdx.z * cs.a;
  __shared__ cx<T> buf[K1_TP * LD];
  __shared__ cx<T> tw[P];
  __shared__ double2 e12[2][K1_TP];
  __shared__ double2 e3[2][MN1];
  const int n1 = N - 1, h = N / 2, nn = n1 * n1, PL = 2 * N - 3;
  const int c0 = blockIdx.x * K1_TP;
  if (c0 >= nn) return;   // a block of the grid's padding (xcd_pencil_blocks)
  const int np = min(K1_TP, nn - c0);
  const int pt = blockIdx.y;
  for (int i = threadIdx.x; i < P; i += NT) tw[i] = twg[i];
  for (int i = threadIdx.x; i < K1_TP * LD; i += NT) buf[i] = cx<T>{0, 0};
  if (mode == ZINV_PAIRS) {
    const double2* phA = ph + (size_t)(pair0 + 2 * pt) * 3 * PL + (N - 2);
    for (int t = threadIdx.x; t < 2 * np; t += NT) {
      const int w = t / np, p = t - w * np;
      const int c = c0 + p, i2 = c / n1, i1 = c - i2 * n1;
      const double2* pw = phA + w * 3 * PL;
      const cx<double> e = cmul(d2c(pw[-2 * (i1 - h + 1)]), d2c(pw[PL - 2 * (i2 - h + 1)]));
      e12[w][p] = double2{e.x, e.y};
    }
    for (int t = threadIdx.x; t < 2 * n1; t += NT) {
      const int w = t / n1, i3 = t - w * n1;
      e3[w][i3] = phA[w * 3 * PL + 2 * PL - 2 * (i3 - h + 1)];
    }
  }
  __syncthreads();
  staged_copy<cx<T>, K1_TP * MN1, NT>(
      np * n1, [&](int e) { const int i3 = e / np; return fc[(size_t)i3 * nn + c0 + e - i3 * np]; },
      [&](int e, cx<T> f) {
        const int i3 = e / np, p = e - i3 * np;
        const int c = c0 + p;
        const int i2 = c / n1, i1 = c - i2 * n1;
        const int k1 = i1 - h + 1, k2 = i2 - h + 1, k3 = i3 - h + 1;
        cx<T> z;
        if (mode == ZINV_PAIRS) {
          const cx<double> eA = cmul(d2c(e12[0][p]), d2c(e3[0][i3]));
          const cx<double> eB = cmul(d2c(e12[1][p]), d2c(e3[1][i3]));
          // E_A + i E_B
          const cx<T> m = {(T)(eA.x - eB.y), (T)(eA.y + eB.x)};
          z = cmul(f, m);
        } else if (mode == ZINV_GRID_SIGN) {
          z = ((k1 + k2 + k3) & 1) ? cx<T>{-f.x, -f.y} : f;
        } else {
          z = f;
        }
        buf[p * LD + posK(i3, h, P)] = z;
      });
  __syncthreads();
  fft_pencils<T, P, +1, NT, K1_TP>(buf, np, RowAddr{LD}, 1, tw);
  const int na = a_plane(N);
  cx<T>* Aout = A + (size_t)pt * P * na;
  for (int e = threadIdx.x; e < np * P; e += NT) {
    const int z = e / np, p = e - z * np;
    Aout[(size_t)z * na + c0 + p] = buf[p * LD + z];
  }
}

// ------------------------------------------------------------------- plane
template <typename T, int P, int NT>
__global__ __launch_bounds__(NT) void k_plane(const cx<T>* __restrict__ A, cx<T>* __restrict__ B,
                                              const T* __restrict__ fgrid, T* __restrict__ gridout,
                                              const cx<T>* __restrict__ twg, int N, int mode, CellStrides cs) {
  constexpr int LD = P + 1;
  A += blockIdx.z * cs.a;
  if (B) B += blockIdx.z * cs.b;
  if (fgrid) fgrid += blockIdx.z * cs.fg;
  if (gridout) gridout += blockIdx.z * cs.fg;
  __shared__ cx<T> plane[P * LD];
  __shared__ cx<T> tw[P];
  const int n1 = N - 1, h = N / 2, nn = n1 * n1;
  const int z = blockIdx.x, pt = blockIdx.y;
  for (int i = threadIdx.x; i < P; i += NT) tw[i] = twg[i];
  for (int i = threadIdx.x; i < P * LD; i += NT) plane[i] = cx<T>{0, 0};
  __syncthreads();
  const cx<T>* Ain = A + ((size_t)pt * P + z) * a_plane(N);
  for (int c = threadIdx.x; c < nn; c += NT) {
    const int i2 = c / n1, i1 = c - i2 * n1;
    plane[posK(i1, h, P) * LD + posK(i2, h, P)] = Ain[c];
  }
  __syncthreads();
  // inverse along axis 2 (rows; only the N-1 rows that hold modes), then axis 1 (columns)
  fft_pencils<T, P, +1, NT, P>(plane, n1, RowKAddr{LD, h, P}, 1, tw);
  fft_pencils<T, P, +1, NT, P>(plane, P, ColAddr{}, LD, tw);
  if (mode == PLANE_TO_GRID) {
    T* out = gridout + (size_t)z * P * P;
    for (int e = threadIdx.x; e < P * P; e += NT) {
      const int x = e / P, y = e - x * P;
      out[e] = plane[x * LD + y].x;
    }
    return;
  }
  const T* fz = fgrid + (size_t)z * P * P;
  for (int e = threadIdx.x; e < P * P; e += NT) {
    const int x = e / P, y = e - x * P;
    plane[x * LD + y] = cscale(plane[x * LD + y], fz[e]);
  }
  __syncthreads();
  fft_pencils<T, P, -1, NT, P>(plane, P, ColAddr{}, LD, tw);
  fft_pencils<T, P, -1, NT, P>(plane, n1, RowKAddr{LD, h, P}, 1, tw);
  const int nhp = nh_pad(N), cmid = (nn - 1) / 2;
  cx<T>* Bout = B + ((size_t)pt * P + z) * 2 * nhp;
  for (int c = threadIdx.x; c < nn; c += NT) {
    const int i2 = c / n1, i1 = c - i2 * n1;
    const cx<T> v = plane[posK(i1, h, P) * LD + posK(i2, h, P)];
    Bout[fold_slot(c, nn, nhp)] = v;
    if (c == cmid) Bout[nhp + cmid] = v;
  }
}

// -------------------------------------------------------------------- zfwd
template <typename T, int P, int NT>
__global__ __launch_bounds__(NT) void k_zfwd(const cx<T>* __restrict__ B, const T* __restrict__ V,
                                             const double2* __restrict__ ph, const double* __restrict__ cp,
                                             double2* __restrict__ Qpart, const cx<T>* __restrict__ twg,
                                             int N, int pair0, int vpair0, int npt, int S, int first,
                                             CellStrides cs) {
  constexpr int LD = P + 1;
  B += blockIdx.z * cs.b;
  Qpart += blockIdx.z * cs.qp;
  constexpr int TQ = K3_TQ;
  constexpr int ROWS = 2 * TQ;
  constexpr int NMAX = (2 * P) / 3;                       // N for the padded length P
  constexpr int OPT = (TQ * (NMAX - 1) + NT - 1) / NT;
  __shared__ cx<T> buf[ROWS * LD];
  __shared__ cx<T> tw[P];
  const int n1 = N - 1, h = N / 2, nn = n1 * n1, nh = (nn + 1) / 2, PL = 2 * N - 3, nhv = weight_row(N);
  // a tile's weight segment is TQ sizeof(T) bytes of a 128-byte line
  constexpr int LG = 128 / (TQ * (int)sizeof(T)) > 1 ? 128 / (TQ * (int)sizeof(T)) : 1;
  const int c0 = xcd_line_tile<LG>((int)blockIdx.x, (int)gridDim.x) * TQ;
  const int nq = min(TQ, nh - c0);
  const int s = blockIdx.y;
  for (int i = threadIdx.x; i < P; i += NT) tw[i] = twg[i];
  for (int i = threadIdx.x; i < ROWS * LD; i += NT) buf[i] = cx<T>{0, 0};
  double accx[OPT], accy[OPT];
#pragma unroll
  for (int b = 0; b < OPT; ++b) accx[b] = accy[b] = 0.0;
  __syncthreads();
  for (int pt = s; pt < npt; pt += S) {
    const int nhp = nh_pad(N);
    const cx<T>* Bin = B + (size_t)pt * P * 2 * nhp;
    // the tile's 2 nq pencils (nq half-spectrum pencils and their mirrors)
    staged_copy<cx<T>, ROWS * P, NT>(
        2 * nq * P,
        [&](int e) {
          const int z = e / (2 * nq), q = e - z * (2 * nq);
          return Bin[(size_t)z * 2 * nhp + (q < nq ? c0 + q : nhp + c0 + q - nq)];
        },
        [&](int e, cx<T> v) {
          const int z = e / (2 * nq), q = e - z * (2 * nq);
          buf[(q < nq ? q : TQ + q - nq) * LD + z] = v;
        });
    __syncthreads();
    fft_pencils<T, P, -1, NT, ROWS>(buf, ROWS, RowAddr{LD}, 1, tw);
    const int jA = pair0 + 2 * pt, jB = jA + 1;
    const double2* phA = ph + (size_t)jA * 3 * PL + (N - 2);
    const double2* phB = phA + 3 * PL;
    const double cA = cp[jA], cB = cp[jB];
    // output mode o: height i3 = o / TQ, pencil c0 + o % TQ (adjacent lanes
    // take adjacent pencils: coalesced weight reads and partial-sum writes)
#pragma unroll
    for (int b = 0; b < OPT; ++b) {
      const int o = threadIdx.x + b * NT;
      const int i3 = o / TQ, q = o - i3 * TQ;
      if (i3 < n1 && q < nq) {
        const int c = c0 + q;
        const int i2 = c / n1, i1 = c - i2 * n1;
        const int k1 = i1 - h + 1, k2 = i2 - h + 1, k3 = i3 - h + 1;
        const cx<T> w1 = buf[q * LD + posK(i3, h, P)];
        const cx<T> w2 = buf[(TQ + q) * LD + posK(n1 - 1 - i3, h, P)];
        // h_A = (w(k) + conj w(-k))/2,  h_B = (w(k) - conj w(-k))/(2i)
        const cx<double> hA = {0.5 * ((double)w1.x + (double)w2.x), 0.5 * ((double)w1.y - (double)w2.y)};
        const cx<double> hB = {0.5 * ((double)w1.y + (double)w2.y), -0.5 * ((double)w1.x - (double)w2.x)};
        const size_t vi = (size_t)i3 * nhv + c;
        const double vA = cA * (double)V[(size_t)(jA - vpair0) * nhv * n1 + vi];
        const double vB = cB * (double)V[(size_t)(jB - vpair0) * nhv * n1 + vi];
        const cx<double> eA = cmul(cmul(d2c(phA[k1]), d2c(phA[PL + k2])), d2c(phA[2 * PL + k3]));
        const cx<double> eB = cmul(cmul(d2c(phB[k1]), d2c(phB[PL + k2])), d2c(phB[2 * PL + k3]));
        const cx<double> tA = cmul(eA, hA), tB = cmul(eB, hB);
        accx[b] += vA * tA.x + vB * tB.x;
        accy[b] += vA * tA.y + vB * tB.y;
      }
    }
    __syncthreads();
  }
  add_partials<OPT>(Qpart, accx, accy, first, [&](int b) -> long long {
    const int o = threadIdx.x + b * NT;
    const int i3 = o / TQ, q = o - i3 * TQ;
    if (i3 >= n1 || q >= nq) return -1;
    return ((long long)s * n1 + i3) * nh + c0 + q;
  });
}


// ------------------------------------------------- plane in three passes
// At P = 128 and 192 a whole plane (P (P+1) complex values) does not fit LDS,
// so the plane stage of one (pair-two, z) plane runs in three launches through
// the row buffer C[pt][z][i1][y] (the N-1 mode rows i1, P values each):
//   rows:    inverse along axis 2 of the N-1 rows of A            -> C
//   columns: inverse along axis 1, product with f (or the real grid
//            out), forward along axis 1 keeping the N-1 modes      -> C in place
//   rows:    forward along axis 2 keeping the N-1 modes           -> B
// Each pass is the same arithmetic as the one-workgroup plane kernels, in LDS
// Stockham passes over a block of rows or columns.
// (16 rows and 16 columns per workgroup: at 128^3 FP32 the plane takes 25.8 ms
// per 440 pair-twos against 27.6 with 32 columns and 28.0 with 8 rows)
template <typename T>
struct SplitCfg {
  static constexpr int RB = 16;   // rows per workgroup
  static constexpr int CB = 16;   // columns per workgroup
  static constexpr int NT = 256;
};

template <typename T, int P>
__global__ __launch_bounds__(SplitCfg<T>::NT) void k_prow_inv(const cx<T>* __restrict__ A, cx<T>* __restrict__ C,
                                                             const cx<T>* __restrict__ twg, int N, CellStrides cs) {
  constexpr int LD = P + 1, RB = SplitCfg<T>::RB, NT = SplitCfg<T>::NT;
  __shared__ cx<T> buf[RB * LD];
  __shared__ cx<T> tw[P];
  const int n1 = N - 1, h = N / 2, nn = n1 * n1;
  const int nrb = (n1 + RB - 1) / RB;
  const int z = blockIdx.x / nrb, r0 = (blockIdx.x - z * nrb) * RB;
  const int nr = min(RB, n1 - r0);
  const int pt = blockIdx.y;
  A += blockIdx.z * cs.a;
  C += blockIdx.z * cs.pc;
  for (int i = threadIdx.x; i < P; i += NT) tw[i] = twg[i];
  for (int i = threadIdx.x; i < RB * LD; i += NT) buf[i] = cx<T>{0, 0};
  __syncthreads();
  // row i1 = r0 + r holds A[i2 n1 + i1] at position posK(i2)
  const cx<T>* Ain = A + ((size_t)pt * P + z) * a_plane(N) + r0;
  staged_copy<cx<T>, RB * maxN1<P>(), NT>(
      nr * n1, [&](int e) { const int i2 = e / nr; return Ain[(size_t)i2 * n1 + e - i2 * nr]; },
      [&](int e, cx<T> v) { const int i2 = e / nr; buf[(e - i2 * nr) * LD + posK(i2, h, P)] = v; });
  __syncthreads();
  fft_pencils<T, P, +1, NT, RB>(buf, nr, RowAddr{LD}, 1, tw);
  cx<T>* Cout = C + (((size_t)pt * P + z) * n1 + r0) * P;
  for (int e = threadIdx.x; e < nr * P; e += NT) {
    const int r = e / P, y = e - r * P;
    Cout[(size_t)r * P + y] = buf[r * LD + y];
  }
}

template <typename T, int P, int MODE>
__global__ __launch_bounds__(SplitCfg<T>::NT) void k_pcol(cx<T>* __restrict__ C, const T* __restrict__ fgrid,
                                                         T* __restrict__ gridout, const cx<T>* __restrict__ twg, int N,
                                                         CellStrides cs) {
  constexpr int LD = P + 1, CB = SplitCfg<T>::CB, NT = SplitCfg<T>::NT;
  static_assert(P % CB == 0, "column blocks");
  __shared__ cx<T> buf[CB * LD];
  __shared__ cx<T> tw[P];
  const int n1 = N - 1, h = N / 2;
  constexpr int ncb = P / CB;
  const int z = blockIdx.x / ncb, y0 = (blockIdx.x - z * ncb) * CB;
  const int pt = blockIdx.y;
  C += blockIdx.z * cs.pc;
  for (int i = threadIdx.x; i < P; i += NT) tw[i] = twg[i];
  for (int i = threadIdx.x; i < CB * LD; i += NT) buf[i] = cx<T>{0, 0};
  __syncthreads();
  // column y0 + q holds the N-1 rows' values at positions posK(i1)
  cx<T>* Cz = C + ((size_t)pt * P + z) * n1 * P + y0;
  staged_copy<cx<T>, maxN1<P>() * CB, NT>(
      n1 * CB, [&](int e) { return Cz[(size_t)(e / CB) * P + e % CB]; },
      [&](int e, cx<T> v) { buf[(e % CB) * LD + posK(e / CB, h, P)] = v; });
  __syncthreads();
  fft_pencils<T, P, +1, NT, CB>(buf, CB, RowAddr{LD}, 1, tw);
  if constexpr (MODE == PLANE_TO_GRID) {
    T* out = gridout + blockIdx.z * cs.fg + (size_t)z * P * P + y0;
    for (int e = threadIdx.x; e < P * CB; e += NT) {
      const int x = e / CB, q = e - x * CB;
      out[(size_t)x * P + q] = buf[q * LD + x].x;
    }
  } else {
    const T* fz = fgrid + blockIdx.z * cs.fg + (size_t)z * P * P + y0;
    staged_copy<T, P * CB, NT>(
        P * CB, [&](int e) { return fz[(size_t)(e / CB) * P + e % CB]; },
        [&](int e, T f) { cx<T>& v = buf[(e % CB) * LD + e / CB]; v = cscale(v, f); });
    __syncthreads();
    fft_pencils<T, P, -1, NT, CB>(buf, CB, RowAddr{LD}, 1, tw);
    for (int e = threadIdx.x; e < n1 * CB; e += NT) {
      const int k1 = e / CB, q = e - k1 * CB;
      Cz[(size_t)k1 * P + q] = buf[q * LD + posK(k1, h, P)];
    }
  }
}

template <typename T, int P>
__global__ __launch_bounds__(SplitCfg<T>::NT) void k_prow_fwd(const cx<T>* __restrict__ C, cx<T>* __restrict__ B,
                                                             const cx<T>* __restrict__ twg, int N, CellStrides cs) {
  constexpr int LD = P + 1, RB = SplitCfg<T>::RB, NT = SplitCfg<T>::NT;
  __shared__ cx<T> buf[RB * LD];
  __shared__ cx<T> tw[P];
  const int n1 = N - 1, h = N / 2, nn = n1 * n1;
  const int nrb = (n1 + RB - 1) / RB;
  const int z = blockIdx.x / nrb, r0 = (blockIdx.x - z * nrb) * RB;
  const int nr = min(RB, n1 - r0);
  const int pt = blockIdx.y;
  C += blockIdx.z * cs.pc;
  B += blockIdx.z * cs.b;
  for (int i = threadIdx.x; i < P; i += NT) tw[i] = twg[i];
  const cx<T>* Cin = C + (((size_t)pt * P + z) * n1 + r0) * P;
  staged_copy<cx<T>, RB * P, NT>(
      nr * P, [&](int e) { return Cin[e]; }, [&](int e, cx<T> v) { buf[(e / P) * LD + e % P] = v; });
  __syncthreads();
  fft_pencils<T, P, -1, NT, RB>(buf, nr, RowAddr{LD}, 1, tw);
  // row k1 = r0 + r gives the modes c = k2 n1 + k1 of the folded B layout
  const int nhp = nh_pad(N), cmid = (nn - 1) / 2;
  cx<T>* Bout = B + ((size_t)pt * P + z) * 2 * nhp;
  for (int e = threadIdx.x; e < nr * n1; e += NT) {
    const int k2 = e / nr, r = e - k2 * nr;
    const int c = k2 * n1 + r0 + r;
    const cx<T> w = buf[r * LD + posK(k2, h, P)];
    Bout[fold_slot(c, nn, nhp)] = w;
    if (c == cmid) Bout[nhp + cmid] = w;
  }
}

template <typename T, int P>
hipError_t plane_rows_t(const void* A, void* B, const void* fgrid, void* gridout, void* C, const void* tw, int N,
                        int npt, int mode, const CellStrides& cs, hipStream_t st) {
  if (!C || N < 2 || N - 1 > P) return hipErrorInvalidValue;
  using S = SplitCfg<T>;
  const int n1 = N - 1, nrb = (n1 + S::RB - 1) / S::RB;
  const dim3 grow(nrb * P, npt, cs.cells), gcol((P / S::CB) * P, npt, cs.cells);
  hipLaunchKernelGGL((k_prow_inv<T, P>), grow, dim3(S::NT), 0, st, (const cx<T>*)A, (cx<T>*)C, (const cx<T>*)tw, N,
                     cs);
  if (mode == PLANE_TO_GRID) {
    hipLaunchKernelGGL((k_pcol<T, P, PLANE_TO_GRID>), gcol, dim3(S::NT), 0, st, (cx<T>*)C, (const T*)nullptr,
                       (T*)gridout, (const cx<T>*)tw, N, cs);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_pcol<T, P, PLANE_PRODUCT>), gcol, dim3(S::NT), 0, st, (cx<T>*)C, (const T*)fgrid,
                     (T*)nullptr, (const cx<T>*)tw, N, cs);
  hipLaunchKernelGGL((k_prow_fwd<T, P>), grow, dim3(S::NT), 0, st, (const cx<T>*)C, (cx<T>*)B, (const cx<T>*)tw, N,
                     cs);
  return hipGetLastError();
}

// ---------------------------------------------------- register-FFT kernels
// A pencil fits the register file when it has at most 96 FP32 or 48 FP64
// complex values; larger pencils use the LDS kernels above.
template <typename T, int P>
struct RegFit {
  static constexpr bool value = (int)sizeof(T) * P <= 4 * 96;
};

template <int P>
constexpr int padN() { return (2 * P) / 3; }
// lengths that occur as a padded length 3N/2 or as an unpadded grid N
template <int P>
constexpr bool isPad() { return P == 12 || P == 24 || P == 36 || P == 48 || P == 72 || P == 96; }
template <int P>
constexpr bool isGrid() { return P == 8 || P == 16 || P == 24 || P == 32 || P == 48 || P == 64; }

// compile-time position of centred index i in a length-P axis with N modes
template <int N, int P>
__device__ __forceinline__ constexpr int posKc(int i) {
  return i - (N / 2 - 1) >= 0 ? i - (N / 2 - 1) : i - (N / 2 - 1) + P;
}

// modulation (mode ZINV_PAIRS), plain copy or grid sign, then inverse FFT
// along axis 3; one thread per pencil c (i1 fastest).  The body of one
// workgroup (pencil block bx, pair-two pt) of one cell; s3 holds 2(N-1)
// values of LDS.  Also the z-inverse of the mixed-size launch.
template <typename T, int N, int P, int NT, int MODE>
__device__ __forceinline__ void zinv_reg_body(const cx<T>* __restrict__ fc, const double2* __restrict__ ph,
                                              cx<T>* __restrict__ A, int pair0, int bx, int pt, cx<T>* s3, const unsigned tx) {
  constexpr int n1 = N - 1, h = N / 2, nn = n1 * n1, PL = 2 * N - 3;
  // axis-3 factors of the pair-two in LDS, in the compute type (see k_zinv_half)
  const double2* phA = MODE == ZINV_PAIRS ? ph + (size_t)(pair0 + 2 * pt) * 3 * PL + (N - 2) : nullptr;
  const double2* phB = MODE == ZINV_PAIRS ? phA + 3 * PL : nullptr;
  if constexpr (MODE == ZINV_PAIRS) {
    for (int t = tx; t < 2 * n1; t += NT) {
      const int i3 = t < n1 ? t : t - n1;
      s3[t] = to_cx<T>((t < n1 ? phA : phB)[2 * PL - 2 * (i3 - h + 1)]);
    }
    __syncthreads();
  }
  const int c = bx * NT + tx;
  if (c >= nn) return;
  const int i2 = c / n1, i1 = c - i2 * n1;
  const int k1 = i1 - h + 1, k2 = i2 - h + 1;
  cx<T> v[P];
#pragma unroll
  for (int i = 0; i < P; ++i) v[i] = cx<T>{0, 0};
  cx<T> eA12 = {1, 0}, eB12 = {0, 0};
  if constexpr (MODE == ZINV_PAIRS) {
    eA12 = cvt<T>(cmul(d2c(phA[-2 * k1]), d2c(phA[PL - 2 * k2])));
    eB12 = cvt<T>(cmul(d2c(phB[-2 * k1]), d2c(phB[PL - 2 * k2])));
  }
#pragma unroll
  for (int i3 = 0; i3 < n1; ++i3) {
    const int k3 = i3 - h + 1;
    const cx<T> f = fc[(size_t)i3 * nn + c];
    cx<T> z;
    if constexpr (MODE == ZINV_PAIRS) {
      const cx<T> eA = cmul(eA12, s3[i3]);
      const cx<T> eB = cmul(eB12, s3[n1 + i3]);
      const cx<T> m = {eA.x - eB.y, eA.y + eB.x};     // E_A + i E_B
      z = cmul(f, m);
    } else if constexpr (MODE == ZINV_GRID_SIGN) {
      z = ((k1 + k2 + k3) & 1) ? cx<T>{-f.x, -f.y} : f;
    } else {
      z = f;
    }
    v[posKc<N, P>(i3)] = z;
  }
  fft_reg<P, +1>(v);
  constexpr int na = a_plane(N);
  cx<T>* Aout = A + (size_t)pt * P * na + c;
#pragma unroll
  for (int zi = 0; zi < P; ++zi) Aout[(size_t)zi * na] = v[zi];
}

template <typename T, int N, int P, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_zinv_reg(const cx<T>* __restrict__ fc, const double2* __restrict__ ph,
                                                 cx<T>* __restrict__ A, int pair0, CellStrides cs) {
  __shared__ cx<T> s3[MODE == ZINV_PAIRS ? 2 * (N - 1) : 1];
  zinv_reg_body<T, N, P, NT, MODE>(fc + blockIdx.z * cs.fc, ph, A + blockIdx.z * cs.a, pair0, blockIdx.x,
                                   blockIdx.y, s3, threadIdx.x);
}

// The first step of an evaluation in one launch: the compact copy of f (as
// k_ingest) and its inverse transform along axis 3 (as k_zinv_reg in mode
// ZINV_PLAIN, into the slot of pair-two 0); one thread per pencil c.
template <typename T, int N, int P, int NT>
__device__ __forceinline__ void zinv_ingest_body(const double2* __restrict__ f, cx<T>* __restrict__ fc,
                                                 cx<T>* __restrict__ A, int* __restrict__ flag, int bx, const unsigned tx) {
  constexpr int n1 = N - 1, h = N / 2, nn = n1 * n1;
  const int c = bx * NT + tx;
  if (c >= nn) return;
  const int i2 = c / n1, i1 = c - i2 * n1;
  const int a = (i1 - h + 1 + N) % N, b = (i2 - h + 1 + N) % N;
  const double2* __restrict__ fp = f + ((size_t)a * N + b) * N;
  cx<T> v[P];
#pragma unroll
  for (int i = 0; i < P; ++i) v[i] = cx<T>{0, 0};
  bool bad = false;
#pragma unroll
  for (int i3 = 0; i3 < n1; ++i3) {
    const double2 d = fp[(i3 - h + 1 + N) % N];
    bad |= !isfinite(d.x) || !isfinite(d.y);
    const cx<T> x = to_cx<T>(d);
    fc[(size_t)i3 * nn + c] = x;
    v[posKc<N, P>(i3)] = x;
  }
  if (bad && flag) flag[0] = 1;
  fft_reg<P, +1>(v);
  constexpr int na = a_plane(N);
  cx<T>* Aout = A + c;
#pragma unroll
  for (int zi = 0; zi < P; ++zi) Aout[(size_t)zi * na] = v[zi];
}

template <typename T, int N, int P, int NT>
__global__ __launch_bounds__(NT) void k_zinv_ingest(PtrPack fin, cx<T>* __restrict__ fc, cx<T>* __restrict__ A,
                                                    CellStrides cs, int* __restrict__ flag) {
  zinv_ingest_body<T, N, P, NT>((const double2*)fin.p[blockIdx.z], fc + blockIdx.z * cs.fc, A + blockIdx.z * cs.a,
                                flag, blockIdx.x, threadIdx.x);
}

template <typename T, int P>
struct PlaneCfg {
  static constexpr int Z = P == 8 ? 8 : P == 12 ? 12 : P == 16 ? 8 : P == 24 ? 8 : P == 32 ? 4
                         : P == 36 ? 3 : P == 48 ? (sizeof(T) == 4 ? 4 : 2) : P == 64 ? 2
                         : P == 72 ? 2 : 1;
  static constexpr int NT = ((Z * P + 63) / 64) * 64;
};

// Z planes of one pair-two per workgroup; one thread per row (axis 2) or
// column (axis 1) of a plane.  LDS holds the N-1 mode rows of each plane.
// The body of one workgroup (z block bx, pair-two pt) of one cell; sm holds
// PlaneCfg<T, P>::Z (N-1)(P+1) values of LDS.  Also the plane stage of the
// mixed-size launch (with more threads than PlaneCfg<T, P>::NT: the extra
// ones idle).
template <typename T, int N, int P, int MODE>
__device__ __forceinline__ void plane_reg_body(const cx<T>* __restrict__ A, cx<T>* __restrict__ B,
                                               const T* __restrict__ fgrid, T* __restrict__ gridout, int bx, int pt,
                                               cx<T>* sm, const unsigned tx) {
  constexpr int n1 = N - 1, nn = n1 * n1, LD = P + 1;
  constexpr int Z = PlaneCfg<T, P>::Z;
  const int z0 = bx * Z;
  const int tid = tx;
  // rows: inverse along axis 2
  if (tid < Z * n1) {
    const int zz = tid / n1, i1 = tid - zz * n1;
    const cx<T>* Ain = A + ((size_t)pt * P + z0 + zz) * a_plane(N) + i1;
    cx<T> v[P];
#pragma unroll
    for (int i = 0; i < P; ++i) v[i] = cx<T>{0, 0};
#pragma unroll
    for (int i2 = 0; i2 < n1; ++i2) v[posKc<N, P>(i2)] = ld_nt(Ain + (size_t)i2 * n1);
    fft_reg<P, +1>(v);
    cx<T>* row = sm + (zz * n1 + i1) * LD;
#pragma unroll
    for (int y = 0; y < P; ++y) row[y] = v[y];
  }
  __syncthreads();
  // columns: inverse along axis 1, product with f (or output of the grid), forward
  if (tid < Z * P) {
    const int zz = tid / P, y = tid - zz * P;
    const int z = z0 + zz;
    cx<T> v[P];
#pragma unroll
    for (int i = 0; i < P; ++i) v[i] = cx<T>{0, 0};
#pragma unroll
    for (int i1 = 0; i1 < n1; ++i1) v[posKc<N, P>(i1)] = sm[(zz * n1 + i1) * LD + y];
    fft_reg<P, +1>(v);
    if constexpr (MODE == PLANE_TO_GRID) {
      T* out = gridout + (size_t)z * P * P + y;
#pragma unroll
      for (int x = 0; x < P; ++x) out[x * P] = v[x].x;
    } else {
      const T* fz = fgrid + (size_t)z * P * P + y;
#pragma unroll
      for (int x = 0; x < P; ++x) v[x] = cscale(v[x], fz[x * P]);
      fft_reg<P, -1>(v);
#pragma unroll
      for (int k1 = 0; k1 < n1; ++k1) sm[(zz * n1 + k1) * LD + y] = v[posKc<N, P>(k1)];
    }
  }
  if constexpr (MODE == PLANE_TO_GRID) return;
  __syncthreads();
  // rows: forward along axis 2, keep the N-1 modes
  if (tid < Z * n1) {
    const int zz = tid / n1, k1 = tid - zz * n1;
    cx<T> v[P];
    const cx<T>* row = sm + (zz * n1 + k1) * LD;
#pragma unroll
    for (int y = 0; y < P; ++y) v[y] = row[y];
    fft_reg<P, -1>(v);
    constexpr int nhp = ((nn + 1) / 2 + 15) / 16 * 16, cmid = (nn - 1) / 2;
    cx<T>* Bout = B + ((size_t)pt * P + z0 + zz) * 2 * nhp;
#pragma unroll
    for (int k2 = 0; k2 < n1; ++k2) {
      const int c = k2 * n1 + k1;
      const cx<T> w = v[posKc<N, P>(k2)];
      st_nt(Bout + (c <= cmid ? c : nhp + (nn - 1 - c)), w);
      if (c == cmid) st_nt(Bout + nhp + cmid, w);
    }
  }
}

template <typename T, int N, int P, int MODE>
__global__ __launch_bounds__((PlaneCfg<T, P>::NT)) void k_plane_reg(const cx<T>* __restrict__ A,
                                                                  cx<T>* __restrict__ B,
                                                                  const T* __restrict__ fgrid,
                                                                  T* __restrict__ gridout, CellStrides cs) {
  __shared__ cx<T> sm[PlaneCfg<T, P>::Z * (N - 1) * (P + 1)];
  if constexpr (MODE == PLANE_TO_GRID)
    plane_reg_body<T, N, P, MODE>(A + blockIdx.z * cs.a, B, fgrid, gridout + blockIdx.z * cs.fg, blockIdx.x,
                                  blockIdx.y, sm, threadIdx.x);
  else
    plane_reg_body<T, N, P, MODE>(A + blockIdx.z * cs.a, B + blockIdx.z * cs.b, fgrid + blockIdx.z * cs.fg, gridout,
                                  blockIdx.x, blockIdx.y, sm, threadIdx.x);
}


// ----------------------------------- two waves per pencil (FP32, P = 72, 96)
// A whole FP32 pencil of 72 or 96 complex values takes most of the register
// file, which leaves one wave per SIMD and exposes every memory wait.  These
// kernels split each transform between two waves of one workgroup by a
// single decimation step in frequency: the wave of parity PAR computes the
// outputs 2j + PAR with a length-P/2 transform (dft_half_dif).  The parity is
// uniform over a wave, so every wave runs straight-line code with
// compile-time twiddles.
template <int P>
struct HalfCfg {
  static constexpr int Q = P / 2;
  static constexpr int WPP = (P + 63) / 64;   // waves per parity (one lane per column)
  static constexpr int NT = 2 * 64 * WPP;
};

// centred index of position m of a length-P axis holding the N-1 modes
// (m < N/2 or m > P - N/2), or -1 for a zero-padding position
template <int N, int P>
__device__ __forceinline__ constexpr int keptK(int m) {
  return m < N / 2 ? m + N / 2 - 1 : (m > P - N / 2 ? m - P + N / 2 - 1 : -1);
}

// rows (axis 2) inverse: outputs y = 2j + PAR of row i1 into LDS
template <typename T, int N, int P, int PAR>
__device__ __forceinline__ void half_rows_inv(const cx<T>* __restrict__ Ain, cx<T>* row) {
  constexpr int n1 = N - 1, Q = P / 2;
  cx<T> u[Q];
  dft_half_dif<P, +1, PAR>(
      [&](int n) -> cx<T> {
        const int i2 = keptK<N, P>(n);
        return i2 >= 0 ? ld_nt(Ain + (size_t)i2 * n1) : cx<T>{0, 0};
      },
      u);
#pragma unroll
  for (int j = 0; j < Q; ++j) row[2 * j + PAR] = u[j];
}

// column y (axis 1): inverse to the outputs x = 2j + PAR, product with f at
// those x, then the length-P/2 forward transform of this parity's samples:
// E[k] (PAR 0) or w_P^{-k} O[k] (PAR 1) of X[k] = E[k] + w^{-k} O[k]
template <typename T, int N, int P, int PAR>
__device__ __forceinline__ void half_cols(const cx<T>* col, const T* __restrict__ fz, cx<T>* u) {
  constexpr int Q = P / 2, LD = P + 1;
  dft_half_dif<P, +1, PAR>(
      [&](int n) -> cx<T> {
        const int i1 = keptK<N, P>(n);
        return i1 >= 0 ? col[i1 * LD] : cx<T>{0, 0};
      },
      u);
#pragma unroll
  for (int j = 0; j < Q; ++j) u[j] = cscale(u[j], fz[(size_t)(2 * j + PAR) * P]);
  fft_reg<Q, -1>(u);
  if constexpr (PAR == 1) {
#pragma unroll
    for (int k = 1; k < Q; ++k) u[k] = twiddle_mul<P, -1>(u[k], k);
  }
}

// after the exchange: u[i] = X[PAR Q/2 + i], u[Q/2 + i] = X[Q + PAR Q/2 + i];
// the kept ones go to row k1 of the plane
template <typename T, int N, int P, int PAR>
__device__ __forceinline__ void half_cols_store(const cx<T>* u, cx<T>* col) {
  constexpr int Q = P / 2, QH = Q / 2, LD = P + 1;
#pragma unroll
  for (int i = 0; i < QH; ++i) {
    const int k1a = keptK<N, P>(PAR * QH + i);
    if (k1a >= 0) col[k1a * LD] = u[i];
    const int k1b = keptK<N, P>(Q + PAR * QH + i);
    if (k1b >= 0) col[k1b * LD] = u[QH + i];
  }
}

// rows (axis 2) forward: kept outputs of parity PAR of row k1 into B
template <typename T, int N, int P, int PAR>
__device__ __forceinline__ void half_rows_fwd(const cx<T>* row, cx<T>* __restrict__ Bout, int k1) {
  constexpr int n1 = N - 1, nn = n1 * n1, Q = P / 2;
  constexpr int nhp = ((nn + 1) / 2 + 15) / 16 * 16, cmid = (nn - 1) / 2;
  cx<T> u[Q];
  dft_half_dif<P, -1, PAR>([&](int n) -> cx<T> { return row[n]; }, u);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int k2 = keptK<N, P>(2 * j + PAR);
    if (k2 >= 0) {
      const int c = k2 * n1 + k1;
      st_nt(Bout + (c <= cmid ? c : nhp + (nn - 1 - c)), u[j]);
      if (c == cmid) st_nt(Bout + nhp + cmid, u[j]);
    }
  }
}

// The row passes of the plane have only N - 1 rows, one wave's worth: with
// the parity split half of the workgroup's waves would sit idle in them.  At
// P = 96 (four waves) each wave takes one class R of a radix-4 decimation in
// frequency instead (outputs 4j + R, dft_quarter_dif), so all four work.
template <int P>
struct QuarterRows {
  static constexpr bool value = P == 96;
};

// rows (axis 2) inverse, class R of the radix-4 split: outputs y = 4j + R of
// the row whose N-1 modes sit at row[i2] (i2 < N-1) of the LDS plane
template <typename T, int N, int P, int R>
__device__ __forceinline__ void quarter_rows_inv(const cx<T>* row, cx<T>* u) {
  dft_quarter_dif<P, +1, R>(
      [&](int n) -> cx<T> {
        const int i2 = keptK<N, P>(n);
        return i2 >= 0 ? row[i2] : cx<T>{0, 0};
      },
      u);
}

template <typename T, int N, int P, int R>
__device__ __forceinline__ void quarter_rows_fwd(const cx<T>* row, cx<T>* __restrict__ Bout, int k1) {
  constexpr int n1 = N - 1, nn = n1 * n1, Q4 = P / 4;
  constexpr int nhp = ((nn + 1) / 2 + 15) / 16 * 16, cmid = (nn - 1) / 2;
  cx<T> u[Q4];
  dft_quarter_dif<P, -1, R>([&](int n) -> cx<T> { return row[n]; }, u);
#pragma unroll
  for (int j = 0; j < Q4; ++j) {
    const int k2 = keptK<N, P>(4 * j + R);
    if (k2 >= 0) {
      const int c = k2 * n1 + k1;
      st_nt(Bout + (c <= cmid ? c : nhp + (nn - 1 - c)), u[j]);
      if (c == cmid) st_nt(Bout + nhp + cmid, u[j]);
    }
  }
}

// Modulation and inverse FFT along axis 3 with two waves per 64 pencils: both
// waves form the modulated pencil (63 values), the wave of parity PAR
// transforms it to the heights z = 2j + PAR (dft_half_dif).
// The axis-3 factors of the two pairs are the same for every lane: they are
// staged once per workgroup in LDS (sA3, sB3, by i3).  The modulation runs in
// the compute type: the factors are unit complex numbers computed in FP64, and
// one product of two of them rounded to FP32 is as accurate as the FP32 input
// it multiplies.
template <typename T, int N, int P, int PAR>
__device__ __forceinline__ void zinv_half_body(const cx<T>* __restrict__ fcb, unsigned c, const cx<T>* sA3,
                                               const cx<T>* sB3, cx<T> eA12, cx<T> eB12,
                                               cx<T>* __restrict__ Ab) {
  constexpr int nn = (N - 1) * (N - 1), Q = P / 2;
  cx<T> u[Q];
  dft_half_dif<P, +1, PAR>(
      [&](int n) -> cx<T> {
        const int i3 = keptK<N, P>(n);
        if (i3 < 0) return cx<T>{0, 0};
        const cx<T> f = *at32(fcb, c + (unsigned)(i3 * nn));
        const cx<T> eA = cmul(eA12, sA3[i3]);
        const cx<T> eB = cmul(eB12, sB3[i3]);
        const cx<T> m = {eA.x - eB.y, eA.y + eB.x};     // E_A + i E_B
        return cmul(f, m);
      },
      u);
#pragma unroll
  for (int j = 0; j < Q; ++j) *at32(Ab, c + (unsigned)((2 * j + PAR) * a_plane(N))) = u[j];
}

template <typename T, int N, int P>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void k_zinv_half(const cx<T>* __restrict__ fc, const double2* __restrict__ ph,
                                                   cx<T>* __restrict__ A, int pair0, CellStrides cs) {
  constexpr int n1 = N - 1, h = N / 2, nn = n1 * n1, PL = 2 * N - 3;
  static_assert((size_t)P * a_plane(N) * sizeof(cx<T>) < (1ull << 32), "32-bit offsets");
  fc += blockIdx.z * cs.fc;
  A += blockIdx.z * cs.a;
  const int pt = blockIdx.y;
  const double2* phA = ph + (size_t)(pair0 + 2 * pt) * 3 * PL + (N - 2);
  const double2* phB = phA + 3 * PL;
  __shared__ cx<T> s3[2 * n1];   // axis-3 factors of pair A (i3 < n1), then of pair B
  for (int t = threadIdx.x; t < 2 * n1; t += 128) {
    const int i3 = t < n1 ? t : t - n1;
    s3[t] = to_cx<T>((t < n1 ? phA : phB)[2 * PL - 2 * (i3 - h + 1)]);
  }
  __syncthreads();
  const int par = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  if (c >= nn) return;
  const int i2 = c / n1, i1 = c - i2 * n1;
  const int k1 = i1 - h + 1, k2 = i2 - h + 1;
  const cx<T> eA12 = cvt<T>(cmul(d2c(phA[-2 * k1]), d2c(phA[PL - 2 * k2])));
  const cx<T> eB12 = cvt<T>(cmul(d2c(phB[-2 * k1]), d2c(phB[PL - 2 * k2])));
  cx<T>* Ab = A + (size_t)pt * P * a_plane(N);
  if (par == 0) zinv_half_body<T, N, P, 0>(fc, (unsigned)c, s3, s3 + n1, eA12, eB12, Ab);
  else zinv_half_body<T, N, P, 1>(fc, (unsigned)c, s3, s3 + n1, eA12, eB12, Ab);
}

// One (pair-two, z) plane per workgroup, as k_plane_reg (mode PLANE_PRODUCT).
// The column pass assembles the forward transform from its two parities by
// one decimation step in time, X[k] = E[k] + w^{-k} O[k] and
// X[k + P/2] = E[k] - w^{-k} O[k]: parity 0 hands E[k], k >= P/4, to parity 1
// and parity 1 hands w^{-k} O[k], k < P/4, to parity 0 through LDS.
template <typename T, int N, int P>
__global__ __launch_bounds__((HalfCfg<P>::NT)) void k_plane_half(const cx<T>* __restrict__ A,
                                                                 cx<T>* __restrict__ B,
                                                                 const T* __restrict__ fgrid,
                                                                 CellStrides cs) {
  using C = HalfCfg<P>;
  constexpr int n1 = N - 1, nn = n1 * n1, LD = P + 1, Q = C::Q, QH = Q / 2;
  static_assert(Q * P <= n1 * LD, "exchange buffer must fit the plane buffer");
  A += blockIdx.z * cs.a;
  B += blockIdx.z * cs.b;
  fgrid += blockIdx.z * cs.fg;
  __shared__ cx<T> sm[n1 * LD];
  const int z = blockIdx.x, pt = blockIdx.y;
  const int par = __builtin_amdgcn_readfirstlane((int)threadIdx.x / (64 * C::WPP));
  const int l = (int)threadIdx.x - par * 64 * C::WPP;
  constexpr bool quarter = QuarterRows<P>::value;
  static_assert(!quarter || (C::NT == 256 && n1 <= 64), "quarter rows need four waves and one row per lane");
  const int wq = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lq = (int)threadIdx.x & 63;
  if constexpr (quarter) {
    // The plane's modes are read from HBM once, coalesced, into the LDS plane
    // (A[i2 n1 + i1] to row i1, position i2); each of the four waves then
    // forms its class of every row from LDS and, once all have read their
    // inputs, writes it over the row in place.  (Each wave reading the rows
    // from memory itself fetched A about twice over at 64^3.)
    const cx<T>* Ap = A + ((size_t)pt * P + z) * a_plane(N);
    staged_copy<cx<T>, nn, C::NT>(
        nn, [&](int e) { return ld_nt(Ap + e); },
        [&](int e, cx<T> v) {
          const int i2 = e / n1;
          sm[(e - i2 * n1) * LD + i2] = v;
        });
    __syncthreads();
    cx<T> u4[P / 4];
    if (lq < n1) {
      const cx<T>* row = sm + lq * LD;
      if (wq == 0) quarter_rows_inv<T, N, P, 0>(row, u4);
      else if (wq == 1) quarter_rows_inv<T, N, P, 1>(row, u4);
      else if (wq == 2) quarter_rows_inv<T, N, P, 2>(row, u4);
      else quarter_rows_inv<T, N, P, 3>(row, u4);
    }
    __syncthreads();
    if (lq < n1) {
#pragma unroll
      for (int j = 0; j < P / 4; ++j) sm[lq * LD + 4 * j + wq] = u4[j];
    }
  } else if (l < n1) {
    const cx<T>* Ain = A + ((size_t)pt * P + z) * a_plane(N) + l;
    if (par == 0) half_rows_inv<T, N, P, 0>(Ain, sm + l * LD);
    else half_rows_inv<T, N, P, 1>(Ain, sm + l * LD);
  }
  __syncthreads();
  cx<T> u[Q];
  const bool col = l < P;
  if (col) {
    const T* fz = fgrid + (size_t)z * P * P + l;
    if (par == 0) half_cols<T, N, P, 0>(sm + l, fz, u);
    else half_cols<T, N, P, 1>(sm + l, fz, u);
  }
  __syncthreads();
  cx<T>* xa = sm;            // E[QH + i] from parity 0, [i][column]
  cx<T>* xb = sm + QH * P;   // w^{-i} O[i] from parity 1
  if (col) {
    if (par == 0) {
#pragma unroll
      for (int i = 0; i < QH; ++i) xa[i * P + l] = u[QH + i];
    } else {
#pragma unroll
      for (int i = 0; i < QH; ++i) xb[i * P + l] = u[i];
    }
  }
  __syncthreads();
  if (col) {
    if (par == 0) {
#pragma unroll
      for (int i = 0; i < QH; ++i) {
        const cx<T> e = u[i], t = xb[i * P + l];
        u[i] = cadd(e, t);
        u[QH + i] = csub(e, t);
      }
    } else {
#pragma unroll
      for (int i = 0; i < QH; ++i) {
        const cx<T> e = xa[i * P + l], t = u[QH + i];
        u[i] = cadd(e, t);
        u[QH + i] = csub(e, t);
      }
    }
  }
  __syncthreads();
  if (col) {
    if (par == 0) half_cols_store<T, N, P, 0>(u, sm + l);
    else half_cols_store<T, N, P, 1>(u, sm + l);
  }
  __syncthreads();
  cx<T>* Bout = B + ((size_t)pt * P + z) * 2 * (((nn + 1) / 2 + 15) / 16 * 16);
  if constexpr (quarter) {
    if (lq < n1) {
      const cx<T>* row = sm + lq * LD;
      if (wq == 0) quarter_rows_fwd<T, N, P, 0>(row, Bout, lq);
      else if (wq == 1) quarter_rows_fwd<T, N, P, 1>(row, Bout, lq);
      else if (wq == 2) quarter_rows_fwd<T, N, P, 2>(row, Bout, lq);
      else quarter_rows_fwd<T, N, P, 3>(row, Bout, lq);
    }
  } else if (l < n1) {
    if (par == 0) half_rows_fwd<T, N, P, 0>(sm + l * LD, Bout, l);
    else half_rows_fwd<T, N, P, 1>(sm + l * LD, Bout, l);
  }
}

// ------------------------------- the plane by column parity (FP64, P = 96)
// The four-wave FP64 plane of k_plane_half fills 97.8 KB of LDS, one
// workgroup per CU, and each of its barriers then idles the CU.  This kernel
// takes the columns y of the plane in two phases by parity p (y = 2c + p), in
// a half plane of LDS, so that two workgroups share a CU:
// * rows, inverse along axis 2: classes R = p and p + 2 of the radix-4 split
//   give the outputs y = 4j + R, i.e. c = 2j + (R - p) / 2 (waves 0, 1);
// * columns c, axis 1: wave R inverts to the points x = 4i + R of the column,
//   multiplies by f, takes the P/4-point forward transform and twiddles it
//   (quarter_cols);
//   the four classes combine their partials through a separate exchange
//   buffer in three rounds, and the kept outputs go back into column c;
// * rows, forward along axis 2: the P/2-point forward transform over c of
//   this phase, D_p, split four ways (wave R: D_p[4j' + R]).  Phase 0 keeps
//   D_0 in registers; phase 1 forms X[k] = D_0[k] + w^{-k} D_1[k] and
//   X[k + P/2] = D_0[k] - w^{-k} D_1[k] and writes the kept modes.
// Rounding differs from the other plane kernels (another split of the same
// transforms); the result is deterministic.  Measured at 64^3 FP64: plane
// stage 27.0 ms against 32.3 ms for k_plane_half (same loads); the default
// there.
template <typename T, int N, int P, int LDC, int R>
__device__ __forceinline__ void quarter_cols(const cx<T>* col, const T* __restrict__ fz, cx<T>* u) {
  constexpr int Q4 = P / 4;
  dft_quarter_dif<P, +1, R>(
      [&](int n) -> cx<T> {
        const int i1 = keptK<N, P>(n);
        return i1 >= 0 ? col[i1 * LDC] : cx<T>{0, 0};
      },
      u);
#pragma unroll
  for (int j = 0; j < Q4; ++j) u[j] = cscale(u[j], fz[(size_t)(4 * j + R) * P]);
  fft_reg<Q4, -1>(u);
  if constexpr (R > 0) {
#pragma unroll
    for (int k = 1; k < Q4; ++k) u[k] = twiddle_mul<P, -1>(u[k], k * R);
  }
}

// (-i)^e x; e is a constant once the callers' loops are unrolled
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> x, int e) {
  switch (e & 3) {
    case 0: return x;
    case 1: return rot<-1>(x);
    case 2: return cx<T>{-x.x, -x.y};
    default: return rot<+1>(x);
  }
}

// Column pass of class R on column c (valid lanes: col).  With
// u_S[k] = w_P^{-S k} D_S[k] from quarter_cols, the forward transform is
// X[k + (P/4) m] = sum_S (-i)^{S m} u_S[k]; class R forms it for k = R + 4t.
// Round rd exchanges t = 2 rd, 2 rd + 1: slot ((Rt * 2 + tt) * 4 + S) * NC + c
// of xch holds u_S[Rt + 4 (2 rd + tt)].
template <typename T, int N, int P, int NC, int LDC, int R>
__device__ __forceinline__ void split_cols_pass(cx<T>* sm, cx<T>* xch, const T* __restrict__ fz, int c,
                                                bool col) {
  constexpr int Q4 = P / 4, NR = Q4 / 8;   // rounds of two frequencies per class
  static_assert(Q4 % 8 == 0, "two frequencies of each class per round");
  cx<T> u[Q4];
  if (col) quarter_cols<T, N, P, LDC, R>(sm + c, fz, u);
  __syncthreads();   // every column input read before outputs overwrite them
#pragma unroll
  for (int rd = 0; rd < NR; ++rd) {
    if (col) {
#pragma unroll
      for (int Rt = 0; Rt < 4; ++Rt) {
        if (Rt == R) continue;
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) xch[((Rt * 2 + tt) * 4 + R) * NC + c] = u[Rt + 4 * (2 * rd + tt)];
      }
    }
    __syncthreads();
    if (col) {
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) {
        const int k = R + 4 * (2 * rd + tt);
        cx<T> sv[4];
#pragma unroll
        for (int S = 0; S < 4; ++S) sv[S] = S == R ? u[k] : xch[((R * 2 + tt) * 4 + S) * NC + c];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int k1 = keptK<N, P>(k + Q4 * m);
          if (k1 < 0) continue;
          sm[k1 * LDC + c] = cadd(cadd(sv[0], mul_mi(sv[1], m)), cadd(mul_mi(sv[2], 2 * m), mul_mi(sv[3], 3 * m)));
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int N, int P, int PH>
__device__ __forceinline__ void split_phase(const cx<T>* __restrict__ Ain0, cx<T>* __restrict__ Bout,
                                            const T* __restrict__ fz0, cx<T>* sm, cx<T>* xch, int wq, int lq,
                                            cx<T>* d0) {
  constexpr int n1 = N - 1, nn = n1 * n1, NC = P / 2, LDC = NC + 1, Q4 = P / 4, Q8 = NC / 4;
  constexpr int nhp = ((nn + 1) / 2 + 15) / 16 * 16, cmid = (nn - 1) / 2;
  // rows, inverse: classes PH (wave 0) and PH + 2 (wave 1) of the P-point
  // split.  The plane's modes are read once per phase, coalesced, by all four
  // waves into LDS (row i1 at sm[i1 n1 ...], over the half plane and the
  // exchange buffer, which follow each other); the two waves form their
  // classes from there and write them into the half plane once every row has
  // been read.  (Each of the two waves reading the rows from memory itself
  // fetched A twice per phase.)
  staged_copy<cx<T>, nn, 256>(
      nn, [&](int e) { return Ain0[e]; },
      [&](int e, cx<T> v) {
        const int i2 = e / n1;
        sm[(e - i2 * n1) * n1 + i2] = v;
      });
  __syncthreads();
  cx<T> u[Q4];
  if (wq < 2 && lq < n1) {
    const cx<T>* rin = sm + lq * n1;
    auto get = [&](int n) -> cx<T> {
      const int i2 = keptK<N, P>(n);
      return i2 >= 0 ? rin[i2] : cx<T>{0, 0};
    };
    if (wq == 0) dft_quarter_dif<P, +1, PH>(get, u);
    else dft_quarter_dif<P, +1, PH + 2>(get, u);
  }
  __syncthreads();
  if (wq < 2 && lq < n1) {
    cx<T>* row = sm + lq * LDC;
#pragma unroll
    for (int j = 0; j < Q4; ++j) row[2 * j + wq] = u[j];
  }
  __syncthreads();
  // columns c (y = 2c + PH), class wq of the points along axis 1
  {
    const bool col = lq < NC;
    const int c = col ? lq : 0;
    const T* fz = fz0 + 2 * c + PH;
    if (wq == 0) split_cols_pass<T, N, P, NC, LDC, 0>(sm, xch, fz, c, col);
    else if (wq == 1) split_cols_pass<T, N, P, NC, LDC, 1>(sm, xch, fz, c, col);
    else if (wq == 2) split_cols_pass<T, N, P, NC, LDC, 2>(sm, xch, fz, c, col);
    else split_cols_pass<T, N, P, NC, LDC, 3>(sm, xch, fz, c, col);
  }
  // rows, forward over this phase's columns: D_PH[4j' + wq]
  if (lq < n1) {
    const cx<T>* row = sm + lq * LDC;
    auto get = [&](int n) -> cx<T> { return row[n]; };
    auto fwd = [&](auto RC) {
      constexpr int R = decltype(RC)::value;
      cx<T> d[Q8];
      dft_quarter_dif<NC, -1, R>(get, d);
      if constexpr (PH == 0) {
#pragma unroll
        for (int j = 0; j < Q8; ++j) d0[j] = d[j];
      } else {
#pragma unroll
        for (int j = 0; j < Q8; ++j) {
          const int k = 4 * j + R;
          const cx<T> b = twiddle_mul<P, -1>(d[j], k);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int k2 = keptK<N, P>(k + h * NC);
            if (k2 < 0) continue;
            const cx<T> w = h == 0 ? cadd(d0[j], b) : csub(d0[j], b);
            const int cc = k2 * n1 + lq;
            st_nt(Bout + (cc <= cmid ? cc : nhp + (nn - 1 - cc)), w);
            if (cc == cmid) st_nt(Bout + nhp + cmid, w);
          }
        }
      }
    };
    if (wq == 0) fwd(std::integral_constant<int, 0>{});
    else if (wq == 1) fwd(std::integral_constant<int, 1>{});
    else if (wq == 2) fwd(std::integral_constant<int, 2>{});
    else fwd(std::integral_constant<int, 3>{});
  }
  __syncthreads();   // the half plane is free for the next phase
}

template <typename T, int N, int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_plane_split(
    const cx<T>* __restrict__ A, cx<T>* __restrict__ B, const T* __restrict__ fgrid, CellStrides cs) {
  constexpr int n1 = N - 1, nn = n1 * n1, NC = P / 2, LDC = NC + 1;
  static_assert(P == 96 && n1 <= 64 && NC <= 64, "one row or column per lane");
  A += blockIdx.z * cs.a;
  B += blockIdx.z * cs.b;
  fgrid += blockIdx.z * cs.fg;
  // the half plane, then the exchange buffer, in one array: together they also
  // hold the plane's n1 x n1 modes staged at the start of each phase
  __shared__ cx<T> lds[n1 * LDC + 4 * 2 * 4 * NC];
  static_assert(n1 * n1 <= n1 * LDC + 4 * 2 * 4 * NC, "staged modes fit");
  cx<T>* sm = lds;
  cx<T>* xch = lds + n1 * LDC;
  const int z = blockIdx.x, pt = blockIdx.y;
  const int wq = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lq = (int)threadIdx.x & 63;
  const cx<T>* Ain = A + ((size_t)pt * P + z) * a_plane(N);
  cx<T>* Bout = B + ((size_t)pt * P + z) * 2 * (((nn + 1) / 2 + 15) / 16 * 16);
  const T* fz = fgrid + (size_t)z * P * P;
  cx<T> d0[NC / 4];
  split_phase<T, N, P, 0>(Ain, Bout, fz, sm, xch, wq, lq, d0);
  split_phase<T, N, P, 1>(Ain, Bout, fz, sm, xch, wq, lq, d0);
}

// The two-dimensional operator (d = 2) at P = 96 in FP32 (FP64 takes
// k_collide2d_split) with the passes of
// k_plane_half: workgroup s carries pair-two s through the whole pipeline in
// one plane of LDS (one pair-two per workgroup: with a loop over several the
// compiler keeps the loop-invariant addresses of every pass in registers and
// spills).  Per pair-two: the y-factors of the two
// pairs' phases staged in LDS; the four-way inverse row passes (axis 2) with
// the modulation f_m (E_A(m) + i E_B(m)) formed on load; the two-parity
// column pass (axis 1: inverse, product with f on the grid, forward, kept
// modes); the four-way forward row passes, whose kept outputs go back into
// their row after every row has been read; then the split of the two pairs,
// the weights and the FP64 accumulation of the half-spectrum modes, as in the
// LDS kernel of the 2-D path.  Layouts as there: compact spectra with mode
// c = i2 (N-1) + i1, f on the grid [x][y], phases ph[pair][axis][2N-3].
template <typename T, int N>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_collide2d_reg(const cx<T>* __restrict__ fc, const T* __restrict__ fgrid,
                                                       const T* __restrict__ V, const double2* __restrict__ ph,
                                                       const double* __restrict__ cp, double2* __restrict__ Qpart,
                                                       int npt, int S) {
  constexpr int P = 3 * N / 2, n1 = N - 1, h = N / 2, nn = n1 * n1, nh = (nn + 1) / 2, PL = 2 * N - 3;
  constexpr int LD = P + 1, Q = P / 2, QH = Q / 2, Q4 = P / 4;
  constexpr int OPT = (nh + 255) / 256;
  static_assert(P == 96 && HalfCfg<P>::NT == 256 && n1 <= 64, "four waves, one row per lane");
  static_assert(sizeof(T) == 4, "FP64 takes k_collide2d_split");
  __shared__ cx<T> sm[n1 * LD];
  __shared__ cx<T> ey[2][n1];
  const int s = blockIdx.x;
  const int par = __builtin_amdgcn_readfirstlane((int)threadIdx.x / 128);
  const int l = (int)threadIdx.x - par * 128;
  const int wq = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lq = (int)threadIdx.x & 63;
  // the pair-two's contribution is this workgroup's row of Qpart
  double2* __restrict__ Qs = Qpart + (size_t)s * nh;
  if (s >= npt) {   // uniform over the workgroup
    for (int c = threadIdx.x; c < nh; c += 256) Qs[c] = double2{0.0, 0.0};
    return;
  }
  {
    const int pt = s;
    const int jA = 2 * pt, jB = jA + 1;
    const double2* phA = ph + (size_t)jA * 2 * PL + (N - 2);
    const double2* phB = phA + 2 * PL;
    for (int t = threadIdx.x; t < 2 * n1; t += 256) {
      const int i2 = t < n1 ? t : t - n1;
      ey[t < n1 ? 0 : 1][i2] = to_cx<T>((t < n1 ? phA : phB)[PL - 2 * (i2 - h + 1)]);
    }
    __syncthreads();
    // the modulated spectrum into the plane: row i1, column i2 (compact)
#pragma unroll 2
    for (int c = threadIdx.x; c < nn; c += 256) {
      const int i2 = c / n1, i1 = c - i2 * n1;
      const int k1 = i1 - h + 1;
      const cx<T> eA = cmul(to_cx<T>(phA[-2 * k1]), ey[0][i2]), eB = cmul(to_cx<T>(phB[-2 * k1]), ey[1][i2]);
      sm[i1 * LD + i2] = cmul(fc[c], cx<T>{eA.x - eB.y, eA.y + eB.x});
    }
    __syncthreads();
    // rows: inverse along axis 2, row i1 = lq; every row is read before any output is written back
    {
      cx<T> u[Q4];
      const cx<T>* row = sm + lq * LD;
      auto get = [&](int n) -> cx<T> {
        const int i2 = keptK<N, P>(n);
        return i2 >= 0 ? row[i2] : cx<T>{0, 0};
      };
      if (lq < n1) {
        if (wq == 0) dft_quarter_dif<P, +1, 0>(get, u);
        else if (wq == 1) dft_quarter_dif<P, +1, 1>(get, u);
        else if (wq == 2) dft_quarter_dif<P, +1, 2>(get, u);
        else dft_quarter_dif<P, +1, 3>(get, u);
      }
      __syncthreads();
      if (lq < n1) {
        cx<T>* out = sm + lq * LD;
        const int R = wq;
#pragma unroll
        for (int j = 0; j < Q4; ++j) out[4 * j + R] = u[j];
      }
    }
    __syncthreads();
    // columns (axis 1): as in k_plane_half
    {
      cx<T> u[Q];
      const bool col = l < P;
      if (col) {
        const T* fz = fgrid + l;
        if (par == 0) half_cols<T, N, P, 0>(sm + l, fz, u);
        else half_cols<T, N, P, 1>(sm + l, fz, u);
      }
      __syncthreads();
      cx<T>* xa = sm;
      cx<T>* xb = sm + QH * P;
      if (col) {
        if (par == 0) {
#pragma unroll
          for (int i = 0; i < QH; ++i) xa[i * P + l] = u[QH + i];
        } else {
#pragma unroll
          for (int i = 0; i < QH; ++i) xb[i * P + l] = u[i];
        }
      }
      __syncthreads();
      if (col) {
        if (par == 0) {
#pragma unroll
          for (int i = 0; i < QH; ++i) {
            const cx<T> e = u[i], t = xb[i * P + l];
            u[i] = cadd(e, t);
            u[QH + i] = csub(e, t);
          }
        } else {
#pragma unroll
          for (int i = 0; i < QH; ++i) {
            const cx<T> e = xa[i * P + l], t = u[QH + i];
            u[i] = cadd(e, t);
            u[QH + i] = csub(e, t);
          }
        }
      }
      __syncthreads();
      if (col) {
        if (par == 0) half_cols_store<T, N, P, 0>(u, sm + l);
        else half_cols_store<T, N, P, 1>(u, sm + l);
      }
      __syncthreads();
    }
    // rows: forward along axis 2; every row is read before any output is written back
    {
      cx<T> u[Q4];
      const cx<T>* row = sm + lq * LD;
      auto get = [&](int n) -> cx<T> { return row[n]; };
      if (lq < n1) {
        if (wq == 0) dft_quarter_dif<P, -1, 0>(get, u);
        else if (wq == 1) dft_quarter_dif<P, -1, 1>(get, u);
        else if (wq == 2) dft_quarter_dif<P, -1, 2>(get, u);
        else dft_quarter_dif<P, -1, 3>(get, u);
      }
      __syncthreads();
      if (lq < n1) {
        cx<T>* out = sm + lq * LD;
        if (wq == 0) {
#pragma unroll
          for (int j = 0; j < Q4; ++j) if (keptK<N, P>(4 * j) >= 0) out[keptK<N, P>(4 * j)] = u[j];
        } else if (wq == 1) {
#pragma unroll
          for (int j = 0; j < Q4; ++j) if (keptK<N, P>(4 * j + 1) >= 0) out[keptK<N, P>(4 * j + 1)] = u[j];
        } else if (wq == 2) {
#pragma unroll
          for (int j = 0; j < Q4; ++j) if (keptK<N, P>(4 * j + 2) >= 0) out[keptK<N, P>(4 * j + 2)] = u[j];
        } else {
#pragma unroll
          for (int j = 0; j < Q4; ++j) if (keptK<N, P>(4 * j + 3) >= 0) out[keptK<N, P>(4 * j + 3)] = u[j];
        }
      }
      __syncthreads();
    }
    // the two pairs, the weights and the accumulation; mode (i1, i2) is sm[i1][i2]
    // (two modes per thread at a time: unrolled fully, the loads of all eight
    // would be hoisted and need more registers than the transforms)
    const double cA = cp[jA], cB = cp[jB];
#pragma unroll 2
    for (int b = 0; b < OPT; ++b) {
      const int c = threadIdx.x + b * 256;
      if (c < nh) {
        const int i2 = c / n1, i1 = c - i2 * n1;
        const int k1 = i1 - h + 1, k2 = i2 - h + 1;
        const cx<T> w1 = sm[i1 * LD + i2];
        const cx<T> w2 = sm[(n1 - 1 - i1) * LD + (n1 - 1 - i2)];
        // h_A = (w(k) + conj w(-k))/2,  h_B = (w(k) - conj w(-k))/(2i)
        const cx<double> hA = {0.5 * ((double)w1.x + (double)w2.x), 0.5 * ((double)w1.y - (double)w2.y)};
        const cx<double> hB = {0.5 * ((double)w1.y + (double)w2.y), -0.5 * ((double)w1.x - (double)w2.x)};
        const double vA = cA * (double)V[(size_t)jA * nh + c];
        const double vB = cB * (double)V[(size_t)jB * nh + c];
        const cx<double> eA = cmul(d2c(phA[k1]), d2c(phA[PL + k2]));
        const cx<double> eB = cmul(d2c(phB[k1]), d2c(phB[PL + k2]));
        const cx<double> tA = cmul(eA, hA), tB = cmul(eB, hB);
        Qs[c] = double2{0.0 + (vA * tA.x + vB * tB.x), 0.0 + (vA * tA.y + vB * tB.y)};
      }
    }
  }
}

// One parity phase of k_collide2d_split (columns y = 2c + PH): rows inverse
// from the modulated spectrum (classes PH, PH + 2 on waves 0, 1), the four-way
// column pass, and the rows forward over this phase's columns (D_PH, class
// wq); phase 0 keeps D_0 in d0, phase 1 forms the kept modes into xo.
template <typename T, int N, int PH>
__device__ __forceinline__ void collide2d_phase(const cx<T>* __restrict__ fc, const T* __restrict__ fgrid,
                                                cx<T>* sm, cx<T>* xch, const cx<T> (*ey)[N - 1], cx<T> pA1,
                                                cx<T> pB1, int wq, int lq, cx<T>* d0, cx<T>* xo) {
  constexpr int P = 3 * N / 2, n1 = N - 1, NC = P / 2, LDC = NC + 1, Q4 = P / 4, Q8 = NC / 4;
  if (wq < 2 && lq < n1) {
    cx<T> u[Q4];
    auto get = [&](int n) -> cx<T> {
      const int i2 = keptK<N, P>(n);
      if (i2 < 0) return cx<T>{0, 0};
      const cx<T> eA = cmul(pA1, ey[0][i2]), eB = cmul(pB1, ey[1][i2]);
      return cmul(fc[i2 * n1 + lq], cx<T>{eA.x - eB.y, eA.y + eB.x});
    };
    cx<T>* row = sm + lq * LDC;
    if (wq == 0) {
      dft_quarter_dif<P, +1, PH>(get, u);
#pragma unroll
      for (int j = 0; j < Q4; ++j) row[2 * j] = u[j];
    } else {
      dft_quarter_dif<P, +1, PH + 2>(get, u);
#pragma unroll
      for (int j = 0; j < Q4; ++j) row[2 * j + 1] = u[j];
    }
  }
  __syncthreads();
  {
    const bool col = lq < NC;
    const int c = col ? lq : 0;
    const T* fz = fgrid + 2 * c + PH;
    if (wq == 0) split_cols_pass<T, N, P, NC, LDC, 0>(sm, xch, fz, c, col);
    else if (wq == 1) split_cols_pass<T, N, P, NC, LDC, 1>(sm, xch, fz, c, col);
    else if (wq == 2) split_cols_pass<T, N, P, NC, LDC, 2>(sm, xch, fz, c, col);
    else split_cols_pass<T, N, P, NC, LDC, 3>(sm, xch, fz, c, col);
  }
  if (lq < n1) {
    const cx<T>* row = sm + lq * LDC;
    auto get = [&](int n) -> cx<T> { return row[n]; };
    auto fwd = [&](auto RC) {
      constexpr int R = decltype(RC)::value;
      cx<T> d[Q8];
      dft_quarter_dif<NC, -1, R>(get, d);
      if constexpr (PH == 0) {
#pragma unroll
        for (int j = 0; j < Q8; ++j) d0[j] = d[j];
      } else {
#pragma unroll
        for (int j = 0; j < Q8; ++j) {
          const cx<T> b = twiddle_mul<P, -1>(d[j], 4 * j + R);
          xo[2 * j] = cadd(d0[j], b);
          xo[2 * j + 1] = csub(d0[j], b);
        }
      }
    };
    if (wq == 0) fwd(std::integral_constant<int, 0>{});
    else if (wq == 1) fwd(std::integral_constant<int, 1>{});
    else if (wq == 2) fwd(std::integral_constant<int, 2>{});
    else fwd(std::integral_constant<int, 3>{});
  }
  __syncthreads();
}

// The two-dimensional operator at P = 96 in FP64 with the plane taken by
// column parity, as k_plane_split: the plane of k_collide2d_reg fills 97.8 KB
// of LDS (one workgroup per CU, its 512 workgroups in two rounds); here a half
// plane and the exchange buffer (74 KB) hold two workgroups per CU.  The row
// input is the modulated spectrum, formed on load; after phase 1 the kept
// modes are gathered in the freed LDS as a compact (N-1) x (N-1) plane for the
// split of the two pairs, the weights and the FP64 accumulation, which are
// those of k_collide2d_reg.
template <typename T, int N>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_collide2d_split(
    const cx<T>* __restrict__ fc, const T* __restrict__ fgrid, const T* __restrict__ V,
    const double2* __restrict__ ph, const double* __restrict__ cp, double2* __restrict__ Qpart, int npt, int S) {
  constexpr int P = 3 * N / 2, n1 = N - 1, h = N / 2, nn = n1 * n1, nh = (nn + 1) / 2, PL = 2 * N - 3;
  constexpr int NC = P / 2, LDC = NC + 1, Q8 = NC / 4, OPT = (nh + 255) / 256;
  constexpr int NPL = n1 * LDC, NX = 4 * 2 * 4 * NC;
  static_assert(P == 96 && n1 <= 64 && nn <= NPL + NX, "one row per lane; the compact plane fits the LDS");
  __shared__ cx<T> lds[NPL + NX];
  __shared__ cx<T> ey[2][n1];
  const int s = blockIdx.x;
  const int wq = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lq = (int)threadIdx.x & 63;
  double2* __restrict__ Qs = Qpart + (size_t)s * nh;
  if (s >= npt) {   // uniform over the workgroup
    for (int c = threadIdx.x; c < nh; c += 256) Qs[c] = double2{0.0, 0.0};
    return;
  }
  const int jA = 2 * s, jB = jA + 1;
  const double2* phA = ph + (size_t)jA * 2 * PL + (N - 2);
  const double2* phB = phA + 2 * PL;
  for (int t = threadIdx.x; t < 2 * n1; t += 256) {
    const int i2 = t < n1 ? t : t - n1;
    ey[t < n1 ? 0 : 1][i2] = to_cx<T>((t < n1 ? phA : phB)[PL - 2 * (i2 - h + 1)]);
  }
  __syncthreads();
  const int k1l = (lq < n1 ? lq : 0) - h + 1;
  const cx<T> pA1 = to_cx<T>(phA[-2 * k1l]), pB1 = to_cx<T>(phB[-2 * k1l]);
  cx<T> d0[Q8], xo[2 * Q8];
  collide2d_phase<T, N, 0>(fc, fgrid, lds, lds + NPL, ey, pA1, pB1, wq, lq, d0, xo);
  collide2d_phase<T, N, 1>(fc, fgrid, lds, lds + NPL, ey, pA1, pB1, wq, lq, d0, xo);
  // the kept modes of row i1 = lq, class wq: X[4j + wq] and X[4j + wq + P/2]
  cx<T>* fin = lds;   // mode (i1, i2) at fin[i1 * n1 + i2]
  if (lq < n1) {
    auto put = [&](auto RC) {
      constexpr int R = decltype(RC)::value;
#pragma unroll
      for (int j = 0; j < Q8; ++j) {
        const int ka = keptK<N, P>(4 * j + R), kb = keptK<N, P>(4 * j + R + NC);
        if (ka >= 0) fin[lq * n1 + ka] = xo[2 * j];
        if (kb >= 0) fin[lq * n1 + kb] = xo[2 * j + 1];
      }
    };
    if (wq == 0) put(std::integral_constant<int, 0>{});
    else if (wq == 1) put(std::integral_constant<int, 1>{});
    else if (wq == 2) put(std::integral_constant<int, 2>{});
    else put(std::integral_constant<int, 3>{});
  }
  __syncthreads();
  const double cA = cp[jA], cB = cp[jB];
#pragma unroll 2
  for (int b = 0; b < OPT; ++b) {
    const int c = threadIdx.x + b * 256;
    if (c < nh) {
      const int i2 = c / n1, i1 = c - i2 * n1;
      const int k1 = i1 - h + 1, k2 = i2 - h + 1;
      const cx<T> w1 = fin[i1 * n1 + i2];
      const cx<T> w2 = fin[(n1 - 1 - i1) * n1 + (n1 - 1 - i2)];
      // h_A = (w(k) + conj w(-k))/2,  h_B = (w(k) - conj w(-k))/(2i)
      const cx<double> hA = {0.5 * ((double)w1.x + (double)w2.x), 0.5 * ((double)w1.y - (double)w2.y)};
      const cx<double> hB = {0.5 * ((double)w1.y + (double)w2.y), -0.5 * ((double)w1.x - (double)w2.x)};
      const double vA = cA * (double)V[(size_t)jA * nh + c];
      const double vB = cB * (double)V[(size_t)jB * nh + c];
      const cx<double> eA = cmul(d2c(phA[k1]), d2c(phA[PL + k2]));
      const cx<double> eB = cmul(d2c(phB[k1]), d2c(phB[PL + k2]));
      const cx<double> tA = cmul(eA, hA), tB = cmul(eB, hB);
      Qs[c] = double2{0.0 + (vA * tA.x + vB * tB.x), 0.0 + (vA * tA.y + vB * tB.y)};
    }
  }
}

// Forward FFT along axis 3 with the weighting and accumulation overlapped:
// producer waves transform the tile's 2 TQ pencils (TQ half-spectrum pencils
// and their mirrors) of pair-two i+1 into one half of a double-buffered LDS
// tile while consumer waves apply the weights of pair-two i from the other
// half and keep their FP64 sums in registers (and fetch the weights of
// pair-two i+1).  One barrier per pair-two (two with two producer waves,
// which hand each other half of their transforms).  A workgroup owns tile
// blockIdx.x and the pair-twos s, s + S, s + 2S ... (s = blockIdx.y).
// Producers: two waves splitting each transform by one decimation step in
// time (P > 48, and FP64 at P = 48; zfwd_dit_*: each wave loads half of the
// heights), or one wave with whole register transforms (FP32 at P <= 48: at
// 32^3 two waves took 0.113 ms against 0.087, while in FP64 they took 0.165
// against 0.176).
template <typename T, int P>
struct ZfwdPipeCfg {
  static constexpr int TQ = 32;
  static constexpr int PW = P > 48 || (P == 48 && sizeof(T) == 8) ? 2 : 1;
  // consumer waves: one at P = 48 (smaller workgroups, more of them per CU:
  // 0.113 -> 0.098 ms at 32^3 FP32), two at P = 72, 96 (one or three: 1.5x
  // slower at 64^3)
  static constexpr int CW = P > 48 ? 2 : 1;
  static constexpr int NT = 64 * (PW + CW);
};

// one producer wave (P <= 48): the whole transform of the lane's pencil
template <typename T, int N, int P>
__device__ __forceinline__ void zfwd_produce(const cx<T>* __restrict__ Bin, cx<T> (*Wb)[64], int r) {
  constexpr int nhp = (((N - 1) * (N - 1) + 1) / 2 + 15) / 16 * 16;
  cx<T> v[P];
#pragma unroll
  for (int z = 0; z < P; ++z) v[z] = Bin[(size_t)z * 2 * nhp];
  fft_reg<P, -1>(v);
#pragma unroll
  for (int i3 = 0; i3 < N - 1; ++i3) Wb[i3][r] = v[posKc<N, P>(i3)];
}

// Two producer waves by one decimation step in time (P > 48).  Wave W loads
// the heights n = 2m + W of its pencil (P/2 of them) and forms
// F_W = DFT_{P/2}; wave 1 scales F_1[k] by w^k (w = e^{-2 pi i / P}), so that
// X[k] = F_0[k] + F_1[k] and X[k + P/2] = F_0[k] - F_1[k].  Wave 0 owns the
// kept outputs k < N/2, wave 1 the kept k + P/2 > P - N/2.  Before a
// workgroup barrier each wave writes into the other's output slots the half
// that one needs (zfwd_dit_send); after it each reads its slots and writes
// its outputs over them (zfwd_dit_finish).
template <typename T, int N, int P, int W>
__device__ __forceinline__ void zfwd_dit_load(const cx<T>* __restrict__ Bin, cx<T>* u) {
  constexpr int nhp = (((N - 1) * (N - 1) + 1) / 2 + 15) / 16 * 16, Q = P / 2;
#pragma unroll
  for (int m = 0; m < Q; ++m) u[m] = Bin[(size_t)(2 * m + W) * 2 * nhp];
  fft_reg<Q, -1>(u);
  if constexpr (W == 1) {
#pragma unroll
    for (int k = 1; k < Q; ++k) u[k] = twiddle_mul<P, -1>(u[k], k);
  }
}

template <typename T, int N, int P, int W>
__device__ __forceinline__ void zfwd_dit_send(const cx<T>* u, cx<T> (*Wb)[64], int r) {
  constexpr int Q = P / 2, h = N / 2;
  static_assert(Q - h + 1 > 0 && h <= Q, "kept outputs of each half");
  if constexpr (W == 1) {
#pragma unroll
    for (int k = 0; k < h; ++k) Wb[keptK<N, P>(k)][r] = u[k];
  } else {
#pragma unroll
    for (int k = Q - h + 1; k < Q; ++k) Wb[keptK<N, P>(k + Q)][r] = u[k];
  }
}

template <typename T, int N, int P, int W>
__device__ __forceinline__ void zfwd_dit_finish(const cx<T>* u, cx<T> (*Wb)[64], int r) {
  constexpr int Q = P / 2, h = N / 2;
  if constexpr (W == 0) {
#pragma unroll
    for (int k = 0; k < h; ++k) {
      cx<T>& w = Wb[keptK<N, P>(k)][r];
      w = cadd(u[k], w);
    }
  } else {
#pragma unroll
    for (int k = Q - h + 1; k < Q; ++k) {
      cx<T>& w = Wb[keptK<N, P>(k + Q)][r];
      w = csub(w, u[k]);
    }
  }
}

// LDS of one k_zfwd_pipe workgroup
template <typename T, int N, int P>
struct ZfwdPipeLds {
  cx<T> W[2][N - 1][2 * ZfwdPipeCfg<T, P>::TQ];
  double2 E12[2][2][ZfwdPipeCfg<T, P>::TQ];
  double2 E3[2][2][N - 1];
  double CPV[2][2];
};

// The body of one workgroup (tile bx, split s) of one cell; also the last
// stage of the mixed-size launch at P = 48.
template <typename T, int N, int P>
__device__ __forceinline__ void zfwd_pipe_body(const cx<T>* __restrict__ B, const T* __restrict__ V,
                                               const double2* __restrict__ ph, const double* __restrict__ cp,
                                               double2* __restrict__ Qpart, int pair0, int vpair0, int npt, int S,
                                               int first, int bx, int s, ZfwdPipeLds<T, N, P>& L, const unsigned tx) {
  using C = ZfwdPipeCfg<T, P>;
  constexpr int TQ = C::TQ, PW = C::PW, NC = 64 * C::CW;
  constexpr int n1 = N - 1, h = N / 2, nn = n1 * n1, nh = (nn + 1) / 2, PL = 2 * N - 3, nhv = weight_row(N);
  constexpr int nhp = (nh + 15) / 16 * 16;
  constexpr int OPT = (TQ * n1 + NC - 1) / NC;
  auto& W = L.W;
  auto& E12 = L.E12;
  auto& E3 = L.E3;
  auto& CPV = L.CPV;
  const int c0 = bx * TQ;
  const int wv = __builtin_amdgcn_readfirstlane((int)tx >> 6);
  const int lane = tx & 63;
  const int nmine = s < npt ? (npt - 1 - s) / S + 1 : 0;
  if (wv < PW) {
    // ---- producers
    const int r = lane;
    const int q = r < TQ ? r : r - TQ;
    const bool have = c0 + q < nh;
    const int cpen = r < TQ ? c0 + q : nn - 1 - (c0 + q);
    const int slot = r < TQ ? c0 + q : nhp + c0 + q;
    for (int i = 0; i <= nmine; ++i) {
      cx<T> u[PW == 2 ? P / 2 : 1];   // this wave's half transform (PW == 2)
      const int b = i & 1;
      if (i < nmine) {
        const int pt = s + i * S;
        const int jA = pair0 + 2 * pt;
        if (have) {
          const cx<T>* Bin = B + (size_t)pt * P * 2 * nhp + slot;
          if constexpr (PW == 1) {
            zfwd_produce<T, N, P>(Bin, W[b], r);
          } else if (wv == 0) {
            zfwd_dit_load<T, N, P, 0>(Bin, u);
            zfwd_dit_send<T, N, P, 0>(u, W[b], r);
          } else {
            zfwd_dit_load<T, N, P, 1>(Bin, u);
            zfwd_dit_send<T, N, P, 1>(u, W[b], r);
          }
        }
        if (wv == 0) {
          if (r < TQ && have) {
            const int i2 = cpen / n1, i1 = cpen - i2 * n1;
            const int k1 = i1 - h + 1, k2 = i2 - h + 1;
#pragma unroll
            for (int w = 0; w < 2; ++w) {
              const double2* pj = ph + (size_t)(jA + w) * 3 * PL + (N - 2);
              const cx<double> e = cmul(d2c(pj[k1]), d2c(pj[PL + k2]));
              E12[b][w][r] = double2{e.x, e.y};
            }
          }
          if (r < 2) CPV[b][r] = cp[jA + r];
        }
        if (wv == PW - 1) {
          for (int e = r; e < 2 * n1; e += 64) {
            const int w = e / n1, i3 = e - w * n1;
            const double2* pj = ph + (size_t)(jA + w) * 3 * PL + (N - 2);
            E3[b][w][i3] = pj[2 * PL + i3 - h + 1];
          }
        }
      }
      if constexpr (PW == 2) {
        lds_barrier();   // the halves handed over are in LDS
        if (i < nmine && have) {
          if (wv == 0) zfwd_dit_finish<T, N, P, 0>(u, W[b], r);
          else zfwd_dit_finish<T, N, P, 1>(u, W[b], r);
        }
      }
      lds_barrier();
    }
  } else {
    // ---- consumers: output modes o = t + bb NC of the tile (i3 = o / TQ, pencil c0 + o % TQ)
    const int t = (int)tx - 64 * PW;
    double accx[OPT], accy[OPT];
    T va[OPT], vb[OPT];
#pragma unroll
    for (int bb = 0; bb < OPT; ++bb) accx[bb] = accy[bb] = 0.0;
    for (int i = 0; i <= nmine; ++i) {
      if (i > 0) {
        const int b = (i - 1) & 1;
        const double cA = CPV[b][0], cB = CPV[b][1];
#pragma unroll
        for (int bb = 0; bb < OPT; ++bb) {
          const int o = t + bb * NC;
          const int i3 = o / TQ, qq = o - i3 * TQ;
          if (o < TQ * n1 && c0 + qq < nh) {
            const cx<T> w1 = W[b][i3][qq];
            const cx<T> w2 = W[b][n1 - 1 - i3][TQ + qq];
            // h_A = (w(k) + conj w(-k))/2,  h_B = (w(k) - conj w(-k))/(2i)
            const cx<double> hA = {0.5 * ((double)w1.x + (double)w2.x), 0.5 * ((double)w1.y - (double)w2.y)};
            const cx<double> hB = {0.5 * ((double)w1.y + (double)w2.y), -0.5 * ((double)w1.x - (double)w2.x)};
            const double vA = cA * (double)va[bb];
            const double vB = cB * (double)vb[bb];
            const cx<double> eA = cmul(d2c(E12[b][0][qq]), d2c(E3[b][0][i3]));
            const cx<double> eB = cmul(d2c(E12[b][1][qq]), d2c(E3[b][1][i3]));
            const cx<double> tA = cmul(eA, hA), tB = cmul(eB, hB);
            accx[bb] += vA * tA.x + vB * tB.x;
            accy[bb] += vA * tA.y + vB * tB.y;
          }
        }
      }
      if (i < nmine) {
        // weights of the pair-two the producers are transforming now
        const int jA = pair0 + 2 * (s + i * S);
        const T* VA = V + (size_t)(jA - vpair0) * nhv * n1;
        const T* VB = VA + (size_t)nhv * n1;
#pragma unroll
        for (int bb = 0; bb < OPT; ++bb) {
          const int o = t + bb * NC;
          const int i3 = o / TQ, qq = o - i3 * TQ;
          const bool ok = o < TQ * n1 && c0 + qq < nh;
          const size_t vi = (size_t)i3 * nhv + c0 + qq;
          va[bb] = ok ? VA[vi] : T(0);
          vb[bb] = ok ? VB[vi] : T(0);
        }
      }
      if constexpr (PW == 2) lds_barrier();   // the producers' hand-over
      lds_barrier();
    }
    add_partials<OPT>(Qpart, accx, accy, first, [&](int bb) -> long long {
      const int o = t + bb * NC;
      const int i3 = o / TQ, qq = o - i3 * TQ;
      if (!(o < TQ * n1 && c0 + qq < nh)) return -1;
      return ((long long)s * n1 + i3) * nh + c0 + qq;
    });
  }
}

template <typename T, int N, int P>
__global__ __launch_bounds__((ZfwdPipeCfg<T, P>::NT)) void k_zfwd_pipe(
    const cx<T>* __restrict__ B, const T* __restrict__ V, const double2* __restrict__ ph,
    const double* __restrict__ cp, double2* __restrict__ Qpart, int pair0, int vpair0, int npt, int S,
    int first, CellStrides cs) {
  __shared__ ZfwdPipeLds<T, N, P> lds;
  zfwd_pipe_body<T, N, P>(B + blockIdx.z * cs.b, V, ph, cp, Qpart + blockIdx.z * cs.qp, pair0, vpair0, npt, S,
                          first, blockIdx.x, blockIdx.y, lds, threadIdx.x);
}

// Forward FFT along axis 3 with one thread per (pencil, pair-two), then the
// split of the two packed pairs, the weights and the FP64 accumulation.
// A workgroup owns TQ half-spectrum pencils c0..c0+TQ-1 (and their mirrors)
// and walks over groups of PT pair-twos; the kept modes of each transform go
// through LDS to the epilogue threads, which own fixed output modes and keep
// their FP64 sums in registers for the whole launch.
// TQ pencils of T make one 128-byte line of the weight table per mode
template <typename T, int P>
struct ZfwdCfg {
  static constexpr int TQ = 128 / (int)sizeof(T);
  static constexpr int PT = sizeof(T) == 4 ? 2 : 4;
  static constexpr int NT = 2 * TQ * PT;
};

// LDS of one k_zfwd_reg workgroup
template <typename T, int N, int P>
struct ZfwdRegLds {
  cx<T> W[ZfwdCfg<T, P>::PT][N - 1][2 * ZfwdCfg<T, P>::TQ];   // kept modes [pt][i3][pencil]
  double2 E12[ZfwdCfg<T, P>::PT][2][ZfwdCfg<T, P>::TQ];       // e^{ia(k1 s1 + k2 s2)} per pair A/B, pencil
  double2 E3[ZfwdCfg<T, P>::PT][2][N - 1];                    // e^{ia k3 s3} per pair A/B
  double CPV[ZfwdCfg<T, P>::PT][2];
};

// The body of one workgroup (tile bx, split s) of one cell; also the last
// stage of the mixed-size launch at P < 48.
template <typename T, int N, int P>
__device__ __forceinline__ void zfwd_reg_body(const cx<T>* __restrict__ B, const T* __restrict__ V,
                                              const double2* __restrict__ ph, const double* __restrict__ cp,
                                              double2* __restrict__ Qpart, int pair0, int vpair0, int npt, int S,
                                              int first, int bx, int s, ZfwdRegLds<T, N, P>& L, const unsigned tx) {
  using C = ZfwdCfg<T, P>;
  constexpr int TQ = C::TQ, PT = C::PT, NT = C::NT;
  constexpr int n1 = N - 1, h = N / 2, nn = n1 * n1, nh = (nn + 1) / 2, PL = 2 * N - 3, nhv = weight_row(N);
  constexpr int OPT = (TQ * n1 + NT - 1) / NT;
  auto& W = L.W;
  auto& E12 = L.E12;
  auto& E3 = L.E3;
  auto& CPV = L.CPV;
  const int c0 = bx * TQ;
  const int tid = tx;
  const int ngroups = (npt + PT - 1) / PT;
  double accx[OPT], accy[OPT];
#pragma unroll
  for (int b = 0; b < OPT; ++b) accx[b] = accy[b] = 0.0;
  // this thread's transform: pt slot p, pencil r (r < TQ: c0 + r, else its mirror)
  const int p = tid / (2 * TQ), r = tid - p * 2 * TQ;
  const int q = r < TQ ? r : r - TQ;
  const bool have = c0 + q < nh;
  const int cpen = r < TQ ? c0 + q : nn - 1 - (c0 + q);
  constexpr int nhp = (nh + 15) / 16 * 16;
  const int slot = r < TQ ? c0 + q : nhp + c0 + q;
  for (int g = s; g < ngroups; g += S) {
    const int pt = g * PT + p;
    if (have && pt < npt) {
      cx<T> v[P];
      const cx<T>* Bin = B + (size_t)pt * P * 2 * nhp + slot;
#pragma unroll
      for (int z = 0; z < P; ++z) v[z] = Bin[(size_t)z * 2 * nhp];
      fft_reg<P, -1>(v);
#pragma unroll
      for (int i3 = 0; i3 < n1; ++i3) W[p][i3][r] = v[posKc<N, P>(i3)];
    }
    // stage the phase factors of this group's pairs
    if (pt < npt) {
      const int jA = pair0 + 2 * pt;
      if (r < TQ && have) {
        const int i2 = cpen / n1, i1 = cpen - i2 * n1;
        const int k1 = i1 - h + 1, k2 = i2 - h + 1;
        for (int w = 0; w < 2; ++w) {
          const double2* pj = ph + (size_t)(jA + w) * 3 * PL + (N - 2);
          const cx<double> e = cmul(d2c(pj[k1]), d2c(pj[PL + k2]));
          E12[p][w][r] = double2{e.x, e.y};
        }
      }
      for (int e = r; e < 2 * n1; e += 2 * TQ) {
        const int w = e / n1, i3 = e - w * n1;
        const double2* pj = ph + (size_t)(jA + w) * 3 * PL + (N - 2);
        E3[p][w][i3] = pj[2 * PL + i3 - h + 1];
      }
      if (r < 2) CPV[p][r] = cp[jA + r];
    }
    __syncthreads();
    const int np = min(PT, npt - g * PT);
#pragma unroll
    for (int b = 0; b < OPT; ++b) {
      const int o = tid + b * NT;
      if (o < TQ * n1) {
        const int i3 = o / TQ, qq = o - i3 * TQ;
        const int c = c0 + qq;
        if (c < nh) {
          for (int pp = 0; pp < np; ++pp) {
            const int jA = pair0 + 2 * (g * PT + pp);
            const cx<T> w1 = W[pp][i3][qq];
            const cx<T> w2 = W[pp][n1 - 1 - i3][TQ + qq];
            // h_A = (w(k) + conj w(-k))/2,  h_B = (w(k) - conj w(-k))/(2i)
            const cx<double> hA = {0.5 * ((double)w1.x + (double)w2.x), 0.5 * ((double)w1.y - (double)w2.y)};
            const cx<double> hB = {0.5 * ((double)w1.y + (double)w2.y), -0.5 * ((double)w1.x - (double)w2.x)};
            const size_t vi = (size_t)i3 * nhv + c;
            const double vA = CPV[pp][0] * (double)V[(size_t)(jA - vpair0) * nhv * n1 + vi];
            const double vB = CPV[pp][1] * (double)V[(size_t)(jA + 1 - vpair0) * nhv * n1 + vi];
            const cx<double> eA = cmul(d2c(E12[pp][0][qq]), d2c(E3[pp][0][i3]));
            const cx<double> eB = cmul(d2c(E12[pp][1][qq]), d2c(E3[pp][1][i3]));
            const cx<double> tA = cmul(eA, hA), tB = cmul(eB, hB);
            accx[b] += vA * tA.x + vB * tB.x;
            accy[b] += vA * tA.y + vB * tB.y;
          }
        }
      }
    }
    __syncthreads();
  }
  add_partials<OPT>(Qpart, accx, accy, first, [&](int b) -> long long {
    const int o = tid + b * NT;
    if (o >= TQ * n1) return -1;
    const int i3 = o / TQ, qq = o - i3 * TQ;
    if (c0 + qq >= nh) return -1;
    return ((long long)s * n1 + i3) * nh + c0 + qq;
  });
}

template <typename T, int N, int P>
__global__ __launch_bounds__((ZfwdCfg<T, P>::NT)) void k_zfwd_reg(
    const cx<T>* __restrict__ B, const T* __restrict__ V, const double2* __restrict__ ph,
    const double* __restrict__ cp, double2* __restrict__ Qpart, int pair0, int vpair0, int npt, int S,
    int first, CellStrides cs) {
  __shared__ ZfwdRegLds<T, N, P> lds;
  zfwd_reg_body<T, N, P>(B + blockIdx.z * cs.b, V, ph, cp, Qpart + blockIdx.z * cs.qp, pair0, vpair0, npt, S, first,
                         blockIdx.x, blockIdx.y, lds, threadIdx.x);
}


// ---------------------------------------------------------------- finalize
// Sixteen lanes per half-spectrum mode (c, i3), 16 modes per workgroup: lane
// r (4 per wave, over the 4 waves) sums the partial accumulators s = r, r + 16,
// ...; the first lane of the mode adds the 16 sums in a fixed order and writes
// Q(k) and, conjugated, Q(-k).  The centre pencil (k1 = k2 = 0) is written
// from k3 >= 0 only, so Q(-k) is exactly conj Q(k) everywhere.  The remaining
// workgroups zero the Nyquist planes.
constexpr int kFinModes = 16, kFinLanes = 16;
// The output of one cell's finalisation and its fused update: Q the result,
// F the state, W the stage buffer (FinUpdate for this cell).
struct FinCell {
  double2* Q;
  double2* F;
  double2* W;
  int mode;
  double a;
};

// the fused update at element i where Q = (qx, qy)
__device__ __forceinline__ void fin_update(const FinCell& u, size_t i, double qx, double qy) {
  const double2 x = u.F[i];
  if (u.mode == FIN_STAGE) {
    u.W[i] = double2{x.x + u.a * qx, x.y + u.a * qy};
  } else {
    const double2 y = u.W[i];
    u.F[i] = double2{x.x + u.a * (y.x + qx), x.y + u.a * (y.y + qy)};
  }
}

// Workgroups of one cell's finalisation at N: the half-spectrum blocks, then
// the Nyquist blocks.
__host__ __device__ __forceinline__ int fin_main_blocks(int N) {
  const int nh = ((N - 1) * (N - 1) + 1) / 2;
  return (nh * (N - 1) + kFinModes - 1) / kFinModes;
}
__host__ __device__ __forceinline__ int fin_blocks(int N) {
  return fin_main_blocks(N) + (3 * N * N - 3 * N + 1 + 255) / 256;
}

// The body of workgroup bx of gx of one cell; also the finalisation of the
// mixed-size launch.
__device__ __forceinline__ void finalize_body(const double2* __restrict__ Qpart, int N, int S, const FinCell& u,
                                              int bx, int gx, double2 (*red)[kFinModes], const unsigned tx) {
  const int n1 = N - 1, h = N / 2, nn = n1 * n1, nh = (nn + 1) / 2, cmid = (nn - 1) / 2;
  double2* __restrict__ Q = u.Q;
  const int nmain = nh * n1;
  const int nnyq = 3 * N * N - 3 * N + 1;
  const int slot = tx & (kFinModes - 1);                       // mode within the workgroup
  const int lane = (tx >> 6) * 4 + ((tx >> 4) & 3);  // residue of s, 0..15
  const int nblk_main = (nmain + kFinModes - 1) / kFinModes;
  if (bx < nblk_main) {
    const int e = bx * kFinModes + slot;
    double x = 0.0, y = 0.0;
    if (e < nmain) {
      const int i3 = e / nh, c = e - i3 * nh;
      for (int s = lane; s < S; s += kFinLanes) {
        const double2 v = Qpart[((size_t)s * n1 + i3) * nh + c];
        x += v.x;
        y += v.y;
      }
    }
    red[lane][slot] = double2{x, y};
    __syncthreads();
    if (tx < kFinModes && e < nmain) {
      const int i3 = e / nh, c = e - i3 * nh;
      const int i2 = c / n1, i1 = c - i2 * n1;
      const int k1 = i1 - h + 1, k2 = i2 - h + 1, k3 = i3 - h + 1;
      if (c == cmid && k3 < 0) return;
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int r = 0; r < kFinLanes; ++r) {
        sx += red[r][slot].x;
        sy += red[r][slot].y;
      }
      const int a = (k1 + N) % N, b = (k2 + N) % N, d = (k3 + N) % N;
      const int am = (N - k1) % N, bm = (N - k2) % N, dm = (N - k3) % N;
      const size_t ip = ((size_t)a * N + b) * N + d, im = ((size_t)am * N + bm) * N + dm;
      const bool mirror = k1 != 0 || k2 != 0 || k3 != 0;
      Q[ip] = double2{sx, sy};
      if (mirror) Q[im] = double2{sx, -sy};
      if (u.mode != FIN_NONE) {
        fin_update(u, ip, sx, sy);
        if (mirror) fin_update(u, im, sx, -sy);
      }
    }
    return;
  }
  // Nyquist entries: plane a = h, then b = h (a != h), then d = h (a, b != h)
  for (int r0 = (bx - nblk_main) * 256 + tx; r0 < nnyq; r0 += (gx - nblk_main) * 256) {
    int r = r0, a, b, d;
    if (r < N * N) { a = h; b = r / N; d = r % N; }
    else if ((r -= N * N) < N * (N - 1)) { a = r / N; a += a >= h; b = h; d = r % N; }
    else { r -= N * (N - 1); a = r / (N - 1); a += a >= h; b = r % (N - 1); b += b >= h; d = h; }
    Q[((size_t)a * N + b) * N + d] = double2{0.0, 0.0};
    if (u.mode != FIN_NONE) fin_update(u, ((size_t)a * N + b) * N + d, 0.0, 0.0);
  }
}

__global__ __launch_bounds__(256) void k_finalize(const double2* __restrict__ Qpart, PtrPack qout, int N, int S,
                                                  size_t qp_stride, FinUpdate upd) {
  __shared__ double2 red[kFinLanes][kFinModes];
  const int c = blockIdx.y;
  const FinCell u{(double2*)qout.p[c], (double2*)upd.f.p[c], (double2*)(upd.ws + (size_t)c * upd.wstride), upd.mode,
                  upd.a};
  finalize_body(Qpart + c * qp_stride, N, S, u, blockIdx.x, gridDim.x, red, threadIdx.x);
}

// ------------------------------------------------------------------- table
// coefficients (-1)^{k+1} / (k!)^2, k = 1..16, of (1 - J0(Y))/Y^2 = 1/4 sum_k c_k (Y^2/4)^{k-1}
struct J1mSeries {
  double c[16];
  constexpr J1mSeries() : c{} {
    double fk2 = 1.0;
    for (int k = 1; k <= 16; ++k) {
      fk2 *= (double)k * (double)k;
      c[k - 1] = ((k & 1) ? 1.0 : -1.0) / fk2;
    }
  }
};
__constant__ J1mSeries kJ1m;

// (1 - J0(Y)) / Y^2: power series below Y = 2 (first dropped term < 1e-28), else from j0
__device__ __forceinline__ double j1m(double Y) {
  if (Y < 2.0) {
    const double z = 0.25 * Y * Y;
    double acc = 0.0;
#pragma unroll
    for (int k = 15; k >= 0; --k) acc = acc * z + kJ1m.c[k];
    return 0.25 * acc;
  }
  return (1.0 - j0(Y)) / (Y * Y);
}

template <typename TV>
__global__ void k_table(TV* __restrict__ V, const double* __restrict__ pd, const double* __restrict__ gj,
                        int nj, int N, int npairs) {
  __shared__ double st[256], sw[256];
  for (int i = threadIdx.x; i < nj; i += blockDim.x) {
    st[i] = gj[i];
    sw[i] = gj[nj + i];
  }
  __syncthreads();
  const int n1 = N - 1, h = N / 2, nhv = weight_row(N);
  const size_t per = (size_t)nhv * n1;
  const size_t total = per * npairs;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / per);
    const int rem = (int)(e - (size_t)j * per);
    const int i3 = rem / nhv, c = rem - i3 * nhv;   // c < nhv < (N-1)^2: a mode of K_N
    const int i2 = c / n1, i1 = c - i2 * n1;
    const double k1 = i1 - h + 1, k2 = i2 - h + 1, k3 = i3 - h + 1;
    const double* p = pd + (size_t)j * 8;
    const double a = p[0], sx = p[1], sy = p[2], sz = p[3], scale = p[4];
    const double kd = k1 * sx + k2 * sy + k3 * sz;
    const double cxp = k2 * sz - k3 * sy, cyp = k3 * sx - k1 * sz, czp = k1 * sy - k2 * sx;
    const double x = a * kd;
    const double y = a * sqrt(cxp * cxp + cyp * cyp + czp * czp);
    double W = 0.0;
    if (x != 0.0 || y != 0.0) {
      const double cosx = cos(x);
      for (int i = 0; i < nj; ++i) {
        const double t = st[i];
        const double Y = 2.0 * y * sqrt(t * (1.0 - t));
        const double jm = j1m(Y);
        const double J = 1.0 - Y * Y * jm;
        // [cos(x(1-2t)) J0(Y) - cos x] / t without cancellation
        const double g = 2.0 * sin(x * (1.0 - t)) * (sin(x * t) / t) * J - cosx * 4.0 * y * y * (1.0 - t) * jm;
        W += sw[i] * g;
      }
    }
    V[e] = (TV)(scale * W);
  }
}

// ------------------------------------------------- weights on the fly
// V = 2 w_sigma Re(e^{-ix} F) / P^3 from the series over even l of
// (2l+1) (-1)^{l/2} mu_l j_l(a |k|) P_l(t), t = k.sigma / |k|, rewritten on the
// host as a Chebyshev series sum_k d_k T_k(u) in u = 2 t^2 - 1 and summed by
// Clenshaw's rule (b_k = d_k + 2u b_{k+1} - b_{k+2}: one subtraction and one
// FMA per term, no per-term constants).  One thread per mode (i3, c) holds the
// d_k of its |k|^2 in registers over the run of pairs that share a radial
// node, and advances PB pairs together; the term count, rounded up to a
// multiple of 8, selects a fully unrolled body (no per-term branches).
// blockIdx.y splits the pair range.
// Pairs jb .. jend-1 of one radial node, MTB Chebyshev terms (the node's
// terms rounded up to a multiple of 8; the extra coefficients are 0).
template <typename T, int PB, int MTB>
__device__ __forceinline__ void wgen_run(T* __restrict__ Vc, const double4* __restrict__ cq,
                                         const double4* __restrict__ pdv, int jb, int jend, int j0, int per, int e,
                                         int k1, int k2, int k3, double rinv) {
  double d[MTB];
#pragma unroll
  for (int g = 0; g < MTB / 4; ++g) {
    const double4 v = cq[g];
    d[4 * g] = v.x;
    d[4 * g + 1] = v.y;
    d[4 * g + 2] = v.z;
    d[4 * g + 3] = v.w;
  }
  for (int jg = jb; jg < jend; jg += PB) {
    double u2[PB], b1[PB], b2[PB];
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const double4 v = pdv[min(jg + q, jend - 1)];
      const double t = ((double)k1 * v.x + (double)k2 * v.y + (double)k3 * v.z) * rinv;
      u2[q] = 4.0 * t * t - 2.0;          // 2u
      b1[q] = 0.0;
      b2[q] = 0.0;
    }
#pragma unroll
    for (int k = MTB - 1; k >= 1; --k) {
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const double b0 = fma(u2[q], b1[q], d[k] - b2[q]);
        b2[q] = b1[q];
        b1[q] = b0;
      }
    }
#pragma unroll
    for (int q = 0; q < PB; ++q)
      if (jg + q < jend)
        Vc[(size_t)(jg + q - j0) * per + e] = (T)(pdv[jg + q].w * fma(0.5 * u2[q], b1[q], d[0] - b2[q]));
  }
}

template <typename T, int PB>
__global__ __launch_bounds__(256) void k_wgen(T* __restrict__ Vc, const double* __restrict__ coef,
                                              const double4* __restrict__ pdv, const int* __restrict__ terms,
                                              int mt, int N, int Mh, int nreal, int j0, int nj, int ncoef) {
  const int n1 = N - 1, h = N / 2, nhv = weight_row(N);
  const int per = nhv * n1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per) return;
  const int i3 = e / nhv, c = e - i3 * nhv;   // c < nhv < (N-1)^2: a mode of K_N
  const int i2 = c / n1, i1 = c - i2 * n1;
  const int k1 = i1 - h + 1, k2 = i2 - h + 1, k3 = i3 - h + 1;
  const int n = k1 * k1 + k2 * k2 + k3 * k3;
  const double rinv = n > 0 ? 1.0 / sqrt((double)n) : 0.0;
  // the pair loop is uniform over the wave (k = 0 needs no branch: its
  // coefficients are all zero, so its weights come out exactly 0)
  const int chunk = (nj + gridDim.y - 1) / gridDim.y;
  int j = j0 + blockIdx.y * chunk;
  const int j1 = min(j0 + nj, j + chunk);
  while (j < j1) {
    const int p = __builtin_amdgcn_readfirstlane(j / Mh);
    const int jend = __builtin_amdgcn_readfirstlane(min(j1, (p + 1) * Mh));
    if (j >= nreal) {
      for (; j < jend; ++j) Vc[(size_t)(j - j0) * per + e] = T(0);
      continue;
    }
    const int b8 = __builtin_amdgcn_readfirstlane((terms[p] + 7) >> 3);
    const double4* cq = (const double4*)(coef + ((size_t)p * ncoef + n) * mt);
    switch (b8) {
      case 1: wgen_run<T, PB, 8>(Vc, cq, pdv, j, jend, j0, per, e, k1, k2, k3, rinv); break;
      case 2: wgen_run<T, PB, 16>(Vc, cq, pdv, j, jend, j0, per, e, k1, k2, k3, rinv); break;
      case 3: wgen_run<T, PB, 24>(Vc, cq, pdv, j, jend, j0, per, e, k1, k2, k3, rinv); break;
      case 4: wgen_run<T, PB, 32>(Vc, cq, pdv, j, jend, j0, per, e, k1, k2, k3, rinv); break;
      case 5: wgen_run<T, PB, 40>(Vc, cq, pdv, j, jend, j0, per, e, k1, k2, k3, rinv); break;
      case 6: wgen_run<T, PB, 48>(Vc, cq, pdv, j, jend, j0, per, e, k1, k2, k3, rinv); break;
      case 7: wgen_run<T, PB, 56>(Vc, cq, pdv, j, jend, j0, per, e, k1, k2, k3, rinv); break;
      case 8: wgen_run<T, PB, 64>(Vc, cq, pdv, j, jend, j0, per, e, k1, k2, k3, rinv); break;
      case 9: wgen_run<T, PB, 72>(Vc, cq, pdv, j, jend, j0, per, e, k1, k2, k3, rinv); break;
      default: wgen_run<T, PB, 80>(Vc, cq, pdv, j, jend, j0, per, e, k1, k2, k3, rinv); break;
    }
    j = jend;
  }
}

// -------------------------------------------------------------- utilities
__global__ void k_fill(double* p, double v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_axpy(double* out, const double* x, double a, const double* y, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = x[i] + a * y[i];
}
__global__ void k_heun(double* f, const double* q1, const double* q2, double hh, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    f[i] = f[i] + hh * (q1[i] + q2[i]);
}
__global__ void k_axpy_cells(PtrPack out, PtrPack x, double a, PtrPack y, size_t n) {
  double* o = out.p[blockIdx.y];
  const double* xx = x.p[blockIdx.y];
  const double* yy = y.p[blockIdx.y];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    o[i] = xx[i] + a * yy[i];
}
__global__ void k_heun_cells(PtrPack f, PtrPack q1, PtrPack q2, double hh, size_t n) {
  double* ff = f.p[blockIdx.y];
  const double* a = q1.p[blockIdx.y];
  const double* b = q2.p[blockIdx.y];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    ff[i] = ff[i] + hh * (a[i] + b[i]);
}
__global__ void k_fill_int(int* p, int v, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_finite(const double* x, size_t n, int* flag) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) flag[0] = 1;
}

__global__ __launch_bounds__(256) void k_moments(const double* __restrict__ f, const double* __restrict__ q,
                                                 double fmin, double L, int N, double* __restrict__ part) {
  __shared__ double red[7][256];
  const double hstep = 2.0 * L / N;
  double s[7] = {0, 0, 0, 0, 0, -1e300, 0};
  const int total = N * N * N;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    // layout [z][x][y]: z = axis 3, x = axis 1, y = axis 2
    const int zi = e / (N * N), xi = (e / N) % N, yi = e % N;
    const double v1 = -L + xi * hstep, v2 = -L + yi * hstep, v3 = -L + zi * hstep;
    const double fv = f[e];
    s[0] += fv;
    s[1] += fv * v1;
    s[2] += fv * v2;
    s[3] += fv * v3;
    s[4] += fv * (v1 * v1 + v2 * v2 + v3 * v3);
    s[5] = fmax(s[5], fv);
    if (q != nullptr && fmin >= 0.0 && fv > fmin) s[6] += q[e] * log(fv);
  }
  for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int k = 0; k < 7; ++k) {
        if (k == 5) red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        else red[k][threadIdx.x] += red[k][threadIdx.x + w];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 7; ++k) part[blockIdx.x * 8 + k] = red[k][0];
}

inline int grid_for(size_t n, int nt) {
  size_t g = (n + nt - 1) / nt;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

// ----------------------------------------------------- dispatch on (P, T)
// N for a launch of length P: the padded length (P = 3N/2) or the grid (P = N)
template <typename T, int P, int N>
hipError_t zinv_reg_t(const void* fc, const double* ph, void* A, int pair0, int npt, int mode,
                      const CellStrides& cs, hipStream_t st) {
  constexpr int nn = (N - 1) * (N - 1);
  constexpr int NT = 64;
  dim3 grid(xcd_pencil_blocks((nn + NT - 1) / NT), npt, cs.cells);
  if (mode == ZINV_PAIRS)
    hipLaunchKernelGGL((k_zinv_reg<T, N, P, NT, ZINV_PAIRS>), grid, dim3(NT), 0, st, (const cx<T>*)fc,
                       (const double2*)ph, (cx<T>*)A, pair0, cs);
  else if (mode == ZINV_GRID_SIGN)
    hipLaunchKernelGGL((k_zinv_reg<T, N, P, NT, ZINV_GRID_SIGN>), grid, dim3(NT), 0, st, (const cx<T>*)fc,
                       (const double2*)ph, (cx<T>*)A, pair0, cs);
  else
    hipLaunchKernelGGL((k_zinv_reg<T, N, P, NT, ZINV_PLAIN>), grid, dim3(NT), 0, st, (const cx<T>*)fc,
                       (const double2*)ph, (cx<T>*)A, pair0, cs);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t zinv_ingest_t(const PtrPack& f, void* fc, void* A, int N, const CellStrides& cs, int* flag,
                         hipStream_t st) {
  if constexpr (RegFit<T, P>::value && isPad<P>()) {
    constexpr int NN = padN<P>(), nn = (NN - 1) * (NN - 1), NT = 64;
    if (N != NN) return hipErrorInvalidValue;
    dim3 grid((nn + NT - 1) / NT, 1, cs.cells);
    hipLaunchKernelGGL((k_zinv_ingest<T, NN, P, NT>), grid, dim3(NT), 0, st, f, (cx<T>*)fc, (cx<T>*)A, cs,
                       flag);
    return hipGetLastError();
  }
  return hipErrorNotSupported;
}

template <typename T, int P, int N>
hipError_t plane_reg_t(const void* A, void* B, const void* fgrid, void* gridout, int npt, int mode,
                       const CellStrides& cs, hipStream_t st) {
  using C = PlaneCfg<T, P>;
  dim3 grid(P / C::Z, npt, cs.cells);
  if (mode == PLANE_TO_GRID)
    hipLaunchKernelGGL((k_plane_reg<T, N, P, PLANE_TO_GRID>), grid, dim3(C::NT), 0, st, (const cx<T>*)A,
                       (cx<T>*)B, (const T*)fgrid, (T*)gridout, cs);
  else
    hipLaunchKernelGGL((k_plane_reg<T, N, P, PLANE_PRODUCT>), grid, dim3(C::NT), 0, st, (const cx<T>*)A,
                       (cx<T>*)B, (const T*)fgrid, (T*)gridout, cs);
  return hipGetLastError();
}

template <typename T, int P, int N>
hipError_t plane_half_t(const void* A, void* B, const void* fgrid, int npt, const CellStrides& cs,
                        hipStream_t st) {
  dim3 grid(P, npt, cs.cells);
  hipLaunchKernelGGL((k_plane_half<T, N, P>), grid, dim3(HalfCfg<P>::NT), 0, st, (const cx<T>*)A, (cx<T>*)B,
                     (const T*)fgrid, cs);
  return hipGetLastError();
}

template <typename T, int P, int N>
hipError_t plane_split_t(const void* A, void* B, const void* fgrid, int npt, const CellStrides& cs,
                         hipStream_t st) {
  dim3 grid(P, npt, cs.cells);
  hipLaunchKernelGGL((k_plane_split<T, N, P>), grid, dim3(256), 0, st, (const cx<T>*)A, (cx<T>*)B,
                     (const T*)fgrid, cs);
  return hipGetLastError();
}

// FP32 pencils of 72 and 96 points use the two-wave kernels
// Kernel variants of the three pipeline stages: 1 = one whole pencil per lane
// (register kernels; LDS kernels where a pencil does not fit the register
// file), 2 = two waves per pencil (z-inverse, plane: P = 48, 72, 96) and the
// pipelined z-forward (P = 24 to 96); 3 = the plane by column parity
// (k_plane_split, FP64 at P = 96 only).  0 selects the default below (the
// fastest in measurements at 16^3 to 64^3: the pipelined z-forward at 24^3
// 35.8 vs 41.5 us FP32, 54.6 vs 69.0 us FP64; a tie at 16^3); plans can be
// autotuned to another.
template <int P>
constexpr bool hasTwo() { return P == 48 || P == 72 || P == 96; }
// lengths with the pipelined z-forward (below P = 48 one producer wave with
// whole register transforms)
template <int P>
constexpr bool hasPipe() { return P == 24 || P == 36 || hasTwo<P>(); }
template <typename T, int P>
constexpr int defaultVariant(int stage) {
  if constexpr (sizeof(T) == 4) {
    if (stage == 2) return P == 36 || P == 48 || P == 72 || P == 96 ? 2 : 1;   // z-forward
    if (stage == 1) return P == 96 ? 2 : 1;                          // plane
    return 1;                                                        // z-inverse
  }
  if (stage == 0) return P == 72 || P == 96 ? 2 : 1;                 // FP64 z-inverse
  if (stage == 1) return P == 96 ? 3 : P == 72 ? 2 : 1;               // FP64 plane
  if (stage == 2) return P == 36 || P == 48 || P == 96 ? 2 : 1;      // FP64 z-forward
  return 1;
}

template <typename T, int P>
hipError_t zinv_t(const void* fc, const double* ph, void* A, const void* tw, int N, int pair0, int npt,
                  int mode, int variant, const CellStrides& cs, hipStream_t st) {
  const int v = variant ? variant : defaultVariant<T, P>(0);
  if constexpr (hasTwo<P>())
    if (v == 2 && N == padN<P>() && mode == ZINV_PAIRS) {
      constexpr int NN = padN<P>(), nn = (NN - 1) * (NN - 1);
      dim3 grid(xcd_pencil_blocks((nn + 63) / 64), npt, cs.cells);
      hipLaunchKernelGGL((k_zinv_half<T, NN, P>), grid, dim3(128), 0, st, (const cx<T>*)fc, (const double2*)ph,
                         (cx<T>*)A, pair0, cs);
      return hipGetLastError();
    }
  if constexpr (RegFit<T, P>::value && isPad<P>())
    if (N == padN<P>()) return zinv_reg_t<T, P, padN<P>()>(fc, ph, A, pair0, npt, mode, cs, st);
  if constexpr (RegFit<T, P>::value && isGrid<P>() && sizeof(T) == 8)
    if (N == P) return zinv_reg_t<T, P, P>(fc, ph, A, pair0, npt, mode, cs, st);
  const int nn = (N - 1) * (N - 1);
  dim3 grid(xcd_pencil_blocks((nn + K1_TP - 1) / K1_TP), npt, cs.cells);
  hipLaunchKernelGGL((k_zinv<T, P, NT_SMALL>), grid, dim3(NT_SMALL), 0, st, (const cx<T>*)fc,
                     (const double2*)ph, (cx<T>*)A, (const cx<T>*)tw, N, pair0, mode, cs);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t plane_t(const void* A, void* B, const void* fgrid, void* gridout, const void* tw, int N,
                   int npt, int mode, int variant, const CellStrides& cs, hipStream_t st) {
  const int v = variant ? variant : defaultVariant<T, P>(1);
  if constexpr (hasTwo<P>())
    if (v == 2 && N == padN<P>() && mode == PLANE_PRODUCT) return plane_half_t<T, P, padN<P>()>(A, B, fgrid, npt, cs, st);
  if constexpr (sizeof(T) == 8 && P == 96)
    if (v == 3 && N == padN<P>() && mode == PLANE_PRODUCT) return plane_split_t<T, P, padN<P>()>(A, B, fgrid, npt, cs, st);
  if constexpr (RegFit<T, P>::value && isPad<P>())
    if (N == padN<P>()) return plane_reg_t<T, P, padN<P>()>(A, B, fgrid, gridout, npt, mode, cs, st);
  if constexpr (RegFit<T, P>::value && isGrid<P>() && sizeof(T) == 8)
    if (N == P) return plane_reg_t<T, P, P>(A, B, fgrid, gridout, npt, mode, cs, st);
  constexpr int NT = PlaneThreads<P>::value;
  dim3 grid(P, npt, cs.cells);
  hipLaunchKernelGGL((k_plane<T, P, NT>), grid, dim3(NT), 0, st, (const cx<T>*)A, (cx<T>*)B,
                     (const T*)fgrid, (T*)gridout, (const cx<T>*)tw, N, mode, cs);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t zfwd_t(const void* B, const void* V, const double* ph, const double* cp, double* Qpart,
                  const void* tw, int N, int pair0, int vpair0, int npt, int S, int first, int variant,
                  const CellStrides& cs, hipStream_t st) {
  const int v = variant ? variant : defaultVariant<T, P>(2);
  if constexpr (hasPipe<P>())
    if (v == 2) {
      using C = ZfwdPipeCfg<T, P>;
      constexpr int NN = padN<P>();
      constexpr int nh = ((NN - 1) * (NN - 1) + 1) / 2;
      dim3 grid((nh + C::TQ - 1) / C::TQ, S, cs.cells);
      hipLaunchKernelGGL((k_zfwd_pipe<T, NN, P>), grid, dim3(C::NT), 0, st, (const cx<T>*)B, (const T*)V,
                         (const double2*)ph, cp, (double2*)Qpart, pair0, vpair0, npt, S, first, cs);
      return hipGetLastError();
    }
  if constexpr (RegFit<T, P>::value && isPad<P>()) {
    using C = ZfwdCfg<T, P>;
    constexpr int NN = padN<P>();
    constexpr int nh = ((NN - 1) * (NN - 1) + 1) / 2;
    dim3 grid((nh + C::TQ - 1) / C::TQ, S, cs.cells);
    hipLaunchKernelGGL((k_zfwd_reg<T, NN, P>), grid, dim3(C::NT), 0, st, (const cx<T>*)B, (const T*)V,
                       (const double2*)ph, cp, (double2*)Qpart, pair0, vpair0, npt, S, first, cs);
    return hipGetLastError();
  }
  const int nn = (N - 1) * (N - 1), nh = (nn + 1) / 2;
  dim3 grid((nh + K3_TQ - 1) / K3_TQ, S, cs.cells);
  hipLaunchKernelGGL((k_zfwd<T, P, NT_SMALL>), grid, dim3(NT_SMALL), 0, st, (const cx<T>*)B,
                     (const T*)V, (const double2*)ph, cp, (double2*)Qpart, (const cx<T>*)tw, N, pair0,
                     vpair0, npt, S, first, cs);
  return hipGetLastError();
}

template <typename T, int P>
int zfwd_blocks_t(int variant) {
  const int v = variant ? variant : defaultVariant<T, P>(2);
  int nb = 0;
  hipError_t e = hipSuccess;
  bool done = false;
  if constexpr (hasPipe<P>())
    if (v == 2) {
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void*>(&k_zfwd_pipe<T, padN<P>(), P>), ZfwdPipeCfg<T, P>::NT, 0);
      done = true;
    }
  if constexpr (RegFit<T, P>::value && isPad<P>())
    if (!done) {
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void*>(&k_zfwd_reg<T, padN<P>(), P>), ZfwdCfg<T, P>::NT, 0);
      done = true;
    }
  if (!done)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_zfwd<T, P, NT_SMALL>),
                                                     NT_SMALL, 0);
  return e == hipSuccess ? nb : 0;
}

#define BZQ_ALL_P(X) X(8) X(12) X(16) X(24) X(32) X(36) X(48) X(64) X(72) X(96)
#define BZQ_PAD_P(X) X(12) X(24) X(36) X(48) X(72) X(96)
// lengths whose plane takes the three-pass kernels (P = 192 for N = 128, and
// the unpadded physical grid P = N = 128)
#define BZQ_BIG_P(X) X(128) X(192)

}  // namespace

// ------------------------------------------------- mixed-size launches
// Independent cells of different N (16, 24, 32; FP32 bulk) in one launch per
// pipeline stage: the launch walks a device work table of (cell, workgroup of
// that cell's stage) items, one item per workgroup, whatever the cells' sizes.
// Each item runs the body of the single-cell kernel for the cell's N with the
// same arguments, so every cell's result is bitwise that of the single-cell
// path.  The cells' geometry and buffers come from MixCell descriptors;
// offs[k] is the first item of cell k (offs[n] = the round's item count).
// A persistent variant (a fixed grid looping over items taken from a device
// counter) kept the loop-invariant addresses and constants of all three sizes
// live across its loop: 213 VGPRs in the plane stage and 247 in the last
// stage, against the 157 and 208 of the single-cell kernels, which costs the
// plane stage a third of its resident waves.  One item per workgroup keeps the
// single-cell register counts.
namespace {

template <int ST>
struct MixCfg;
template <>
struct MixCfg<MIX_INGEST> {
  static constexpr int NT = 64;
  static constexpr size_t LDS = 16;
};
template <>
struct MixCfg<MIX_GRID> {
  static constexpr int NT = 192;
  static constexpr size_t LDS = PlaneCfg<float, 48>::Z * 31 * 49 * 8;
};
template <>
struct MixCfg<MIX_ZINV> {
  static constexpr int NT = 64;
  static constexpr size_t LDS = 2 * 31 * 8;
};
template <>
struct MixCfg<MIX_PLANE> {
  static constexpr int NT = 192;
  static constexpr size_t LDS = PlaneCfg<float, 48>::Z * 31 * 49 * 8;
};
template <>
struct MixCfg<MIX_ZFWD> {
  static constexpr int NT = 128;
  static constexpr size_t LDS = sizeof(ZfwdPipeLds<float, 32, 48>) > sizeof(ZfwdRegLds<float, 24, 36>)
                                    ? sizeof(ZfwdPipeLds<float, 32, 48>)
                                    : sizeof(ZfwdRegLds<float, 24, 36>);
};
template <>
struct MixCfg<MIX_FINAL> {
  static constexpr int NT = 256;
  static constexpr size_t LDS = sizeof(double2) * kFinLanes * kFinModes;
};

template <int N>
constexpr int mixP() { return 3 * N / 2; }

// one item of stage ST for a cell of size N; `local` is the item within the cell
template <int ST, int N>
__device__ __forceinline__ void mix_item(const MixCell& c, int local, int phase, double a, double2* const* outs,
                                         unsigned char* lds, const unsigned tx) {
  constexpr int P = mixP<N>(), n1 = N - 1, nn = n1 * n1;
  static_assert(PlaneCfg<float, P>::NT <= MixCfg<MIX_PLANE>::NT, "plane threads");
  const double2* fin = phase == 2 ? c.fs : c.f;
  if constexpr (ST == MIX_INGEST) {
    zinv_ingest_body<float, N, P, 64>(fin, (cx<float>*)c.fc, (cx<float>*)c.A, nullptr, local, tx);
  } else if constexpr (ST == MIX_GRID) {
    plane_reg_body<float, N, P, PLANE_TO_GRID>((const cx<float>*)c.A, nullptr, nullptr, c.fgrid, local, 0,
                                               (cx<float>*)lds, tx);
  } else if constexpr (ST == MIX_ZINV) {
    constexpr int gx = (nn + 63) / 64;
    zinv_reg_body<float, N, P, 64, ZINV_PAIRS>((const cx<float>*)c.fc, c.ph, (cx<float>*)c.A, 0, local % gx, local / gx,
                                               (cx<float>*)lds, tx);
  } else if constexpr (ST == MIX_PLANE) {
    constexpr int gx = P / PlaneCfg<float, P>::Z;
    plane_reg_body<float, N, P, PLANE_PRODUCT>((const cx<float>*)c.A, (cx<float>*)c.B, c.fgrid, nullptr, local % gx,
                                               local / gx, (cx<float>*)lds, tx);
  } else if constexpr (ST == MIX_ZFWD) {
    constexpr int tiles = ((nn + 1) / 2 + 31) / 32;
    if constexpr (P == 48)
      zfwd_pipe_body<float, N, P>((const cx<float>*)c.B, c.V, c.ph, c.cp, c.Qpart, 0, 0, c.npt, c.S, 1, local % tiles,
                                  local / tiles,
                                  *(ZfwdPipeLds<float, N, P>*)lds, tx);
    else
      zfwd_reg_body<float, N, P>((const cx<float>*)c.B, c.V, c.ph, c.cp, c.Qpart, 0, 0, c.npt, c.S, 1, local % tiles,
                                 local / tiles,
                                 *(ZfwdRegLds<float, N, P>*)lds, tx);
  } else {
    FinCell u;
    u.F = c.f;
    if (phase == 0) {
      u.Q = outs[c.cell];
      u.W = nullptr;
      u.mode = FIN_NONE;
    } else if (phase == 1) {
      u.Q = c.q1;
      u.W = c.fs;
      u.mode = FIN_STAGE;
    } else {
      u.Q = c.q2;
      u.W = c.q1;
      u.mode = FIN_HEUN;
    }
    u.a = a;
    finalize_body(c.Qpart, N, c.S, u, local, fin_blocks(N), (double2(*)[kFinModes])lds, tx);
  }
}

template <int ST>
__global__ __launch_bounds__(MixCfg<ST>::NT) void k_mix(const MixCell* __restrict__ cells, const int* __restrict__ offs,
                                                        int ncells, int phase, double a,
                                                        double2* const* __restrict__ outs) {
  __shared__ __align__(16) unsigned char lds[MixCfg<ST>::LDS];
  // the item's cell: the last k with offs[k] <= item (uniform over the workgroup)
  const int item = blockIdx.x;
  int lo = 0, hi = ncells;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offs[mid] <= item) lo = mid;
    else hi = mid;
  }
  const MixCell& c = cells[lo];
  const int local = item - offs[lo];
  if (c.N == 16) mix_item<ST, 16>(c, local, phase, a, outs, lds, threadIdx.x);
  else if (c.N == 24) mix_item<ST, 24>(c, local, phase, a, outs, lds, threadIdx.x);
  else mix_item<ST, 32>(c, local, phase, a, outs, lds, threadIdx.x);
}

template <int ST>
int mix_items_t(int N, int npt, int S) {
  auto per = [&](auto tag) -> int {
    constexpr int NN = decltype(tag)::value, P = mixP<NN>(), nn = (NN - 1) * (NN - 1);
    if constexpr (ST == MIX_INGEST) return (nn + 63) / 64;
    else if constexpr (ST == MIX_GRID) return P / PlaneCfg<float, P>::Z;
    else if constexpr (ST == MIX_ZINV) return (nn + 63) / 64 * npt;
    else if constexpr (ST == MIX_PLANE) return P / PlaneCfg<float, P>::Z * npt;
    else if constexpr (ST == MIX_ZFWD) return ((nn + 1) / 2 + 31) / 32 * S;
    else return fin_blocks(NN);
  };
  if (N == 16) return per(std::integral_constant<int, 16>{});
  if (N == 24) return per(std::integral_constant<int, 24>{});
  if (N == 32) return per(std::integral_constant<int, 32>{});
  return 0;
}

template <int ST>
hipError_t mix_launch_t(const MixCell* cells, const int* offs, int ncells, int total, int phase, double a,
                        double2* const* outs, hipStream_t st) {
  if (total < 1) return hipSuccess;
  hipLaunchKernelGGL(k_mix<ST>, dim3(total), dim3(MixCfg<ST>::NT), 0, st, cells, offs, ncells, phase, a, outs);
  return hipGetLastError();
}

}  // namespace

bool mix_supported(int N, bool fp32, int zinv_variant, int plane_variant, int zfwd_variant) {
  if (!fp32 || (N != 16 && N != 24 && N != 32)) return false;
  return zinv_variant == 1 && plane_variant == 1 && zfwd_variant == (N == 32 ? 2 : 1);
}

int mix_items(int stage, int N, int npt, int S) {
  switch (stage) {
    case MIX_INGEST: return mix_items_t<MIX_INGEST>(N, npt, S);
    case MIX_GRID: return mix_items_t<MIX_GRID>(N, npt, S);
    case MIX_ZINV: return mix_items_t<MIX_ZINV>(N, npt, S);
    case MIX_PLANE: return mix_items_t<MIX_PLANE>(N, npt, S);
    case MIX_ZFWD: return mix_items_t<MIX_ZFWD>(N, npt, S);
    case MIX_FINAL: return mix_items_t<MIX_FINAL>(N, npt, S);
  }
  return 0;
}

hipError_t launch_mix(int stage, const MixCell* cells, const int* offs, int ncells, int total, int phase, double a,
                      double2* const* outs, hipStream_t st) {
  switch (stage) {
    case MIX_INGEST: return mix_launch_t<MIX_INGEST>(cells, offs, ncells, total, phase, a, outs, st);
    case MIX_GRID: return mix_launch_t<MIX_GRID>(cells, offs, ncells, total, phase, a, outs, st);
    case MIX_ZINV: return mix_launch_t<MIX_ZINV>(cells, offs, ncells, total, phase, a, outs, st);
    case MIX_PLANE: return mix_launch_t<MIX_PLANE>(cells, offs, ncells, total, phase, a, outs, st);
    case MIX_ZFWD: return mix_launch_t<MIX_ZFWD>(cells, offs, ncells, total, phase, a, outs, st);
    case MIX_FINAL: return mix_launch_t<MIX_FINAL>(cells, offs, ncells, total, phase, a, outs, st);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------ no-allocation scratch
// The scratch of bzq_collision_noalloc: a file-scope device array, one copy on
// every GPU the library runs on, held until the process ends.  In host code
// the array's name is only a host-side stand-in; the device address comes
// from hipGetSymbolAddress, once per device with that device current, and is
// the only handle host code passes on (kernel arguments, copies).
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptrs[kMaxDevices] = {};
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return hipSuccess;
}


hipError_t launch_ingest(const PtrPack& f, void* fc, size_t fc_stride, int cells, int N, bool fp32,
                         hipStream_t st, int* flag) {
  const size_t n = (size_t)(N - 1) * (N - 1) * (N - 1);
  dim3 grid(grid_for(n, 256), cells);
  if (fp32)
    hipLaunchKernelGGL(k_ingest<float>, grid, dim3(256), 0, st, f, (cx<float>*)fc, fc_stride, N, flag);
  else
    hipLaunchKernelGGL(k_ingest<double>, grid, dim3(256), 0, st, f, (cx<double>*)fc, fc_stride, N, flag);
  return hipGetLastError();
}

// FP32: k_collide2d_reg; FP64: k_collide2d_split (two workgroups per CU; N = 64,
// 512 pair-twos: 0.063 -> 0.058 ms per evaluation against the one-plane kernel)
hipError_t launch_collide2d_reg(const void* fc, const void* fgrid, const void* V, const double* ph, const double* cp,
                                double* Qpart, int N, int npt, int S, bool fp32, hipStream_t st) {
  if (N != 64 || S < npt) return hipErrorInvalidValue;   // one pair-two per workgroup
  if (fp32)
    hipLaunchKernelGGL((k_collide2d_reg<float, 64>), dim3(S), dim3(256), 0, st, (const cx<float>*)fc,
                       (const float*)fgrid, (const float*)V, (const double2*)ph, cp, (double2*)Qpart, npt, S);
  else
    hipLaunchKernelGGL((k_collide2d_split<double, 64>), dim3(S), dim3(256), 0, st, (const cx<double>*)fc,
                       (const double*)fgrid, (const double*)V, (const double2*)ph, cp, (double2*)Qpart, npt, S);
  return hipGetLastError();
}

bool zinv_ingest_fits(int P, bool fp32) {
  return (P == 12 || P == 24 || P == 36 || P == 48 || P == 72 || P == 96) && (fp32 ? 4 : 8) * P <= 4 * 96;
}

hipError_t launch_zinv_ingest(const PtrPack& f, void* fc, void* A, Geometry g, bool fp32, const CellStrides& cs,
                              hipStream_t st, int* flag) {
#define CASE(PP)                                                             \
  case PP:                                                                   \
    return fp32 ? zinv_ingest_t<float, PP>(f, fc, A, g.N, cs, flag, st)      \
                : zinv_ingest_t<double, PP>(f, fc, A, g.N, cs, flag, st);
  switch (g.P) { BZQ_PAD_P(CASE) }
#undef CASE
  return hipErrorInvalidValue;
}

hipError_t launch_zinv(const void* fc, const double* ph, void* A, const void* tw, Geometry g, int pair0,
                       int npt, int mode, bool fp32, const CellStrides& cs, hipStream_t st, int variant) {
#define CASE(PP)                                                                                 \
  case PP:                                                                                       \
    return fp32 ? zinv_t<float, PP>(fc, ph, A, tw, g.N, pair0, npt, mode, variant, cs, st)      \
                : zinv_t<double, PP>(fc, ph, A, tw, g.N, pair0, npt, mode, variant, cs, st);
  switch (g.P) { BZQ_ALL_P(CASE) BZQ_BIG_P(CASE) }
#undef CASE
  return hipErrorInvalidValue;
}

bool needs_plane_rows(int P) { return P == 128 || P == 192; }

hipError_t launch_plane(const void* A, void* B, const void* fgrid, void* gridout, const void* tw,
                        Geometry g, int npt, int mode, bool fp32, const CellStrides& cs, hipStream_t st,
                        int variant, void* C) {
#define CASE(PP)                                                                                   \
  case PP:                                                                                         \
    return fp32 ? plane_t<float, PP>(A, B, fgrid, gridout, tw, g.N, npt, mode, variant, cs, st)   \
                : plane_t<double, PP>(A, B, fgrid, gridout, tw, g.N, npt, mode, variant, cs, st);
  switch (g.P) { BZQ_ALL_P(CASE) }
#undef CASE
#define CASE(PP)                                                                                           \
  case PP:                                                                                                 \
    return fp32 ? plane_rows_t<float, PP>(A, B, fgrid, gridout, C, tw, g.N, npt, mode, cs, st)            \
                : plane_rows_t<double, PP>(A, B, fgrid, gridout, C, tw, g.N, npt, mode, cs, st);
  switch (g.P) { BZQ_BIG_P(CASE) }
#undef CASE
  return hipErrorInvalidValue;
}

hipError_t launch_zfwd(const void* B, const void* V, const double* ph, const double* cp, double* Qpart,
                       const void* tw, Geometry g, int pair0, int npt, int S, bool fp32,
                       const CellStrides& cs, hipStream_t st, int variant, int vpair0, bool first) {
#define CASE(PP)                                                                                      \
  case PP:                                                                                            \
    return fp32 ? zfwd_t<float, PP>(B, V, ph, cp, Qpart, tw, g.N, pair0, vpair0, npt, S, first, variant, cs, st) \
                : zfwd_t<double, PP>(B, V, ph, cp, Qpart, tw, g.N, pair0, vpair0, npt, S, first, variant, cs, st);
  switch (g.P) { BZQ_PAD_P(CASE) CASE(192) }
#undef CASE
  return hipErrorInvalidValue;
}

int zfwd_blocks_per_cu(int P, bool fp32, int variant) {
#define CASE(PP) \
  case PP:       \
    return fp32 ? zfwd_blocks_t<float, PP>(variant) : zfwd_blocks_t<double, PP>(variant);
  switch (P) { BZQ_PAD_P(CASE) }
#undef CASE
  return 0;
}

int stage_default_variant(int stage, int P, bool fp32) {
#define CASE(PP) \
  case PP:       \
    return fp32 ? defaultVariant<float, PP>(stage) : defaultVariant<double, PP>(stage);
  switch (P) { BZQ_ALL_P(CASE) }
#undef CASE
  return 1;
}

unsigned stage_variants(int stage, int P, bool fp32) {
  if (stage == 1 && P == 96 && !fp32) return 0xEu;   // 3: the plane by column parity (k_plane_split)
  if (stage == 2 && (P == 24 || P == 36)) return 0x6u;   // 2: the pipelined z-forward
  return (P == 48 || P == 72 || P == 96) ? 0x6u : 0x2u;
}

hipError_t launch_finalize(const double* Qpart, const PtrPack& Q, size_t qp_stride, int cells, int N, int S,
                           hipStream_t st, const FinUpdate& upd) {
  dim3 grid((unsigned)fin_blocks(N), cells);
  hipLaunchKernelGGL(k_finalize, grid, dim3(256), 0, st, (const double2*)Qpart, Q, N, S, qp_stride, upd);
  return hipGetLastError();
}

hipError_t launch_axpy_cells(const PtrPack& out, const PtrPack& x, double a, const PtrPack& y, size_t n,
                             int cells, hipStream_t st) {
  dim3 grid(grid_for(2 * n, 256), cells);
  hipLaunchKernelGGL(k_axpy_cells, grid, dim3(256), 0, st, out, x, a, y, 2 * n);
  return hipGetLastError();
}
hipError_t launch_heun_cells(const PtrPack& f, const PtrPack& q1, const PtrPack& q2, double hh, size_t n,
                             int cells, hipStream_t st) {
  dim3 grid(grid_for(2 * n, 256), cells);
  hipLaunchKernelGGL(k_heun_cells, grid, dim3(256), 0, st, f, q1, q2, hh, 2 * n);
  return hipGetLastError();
}

hipError_t launch_table(void* V, const double* pd, const double* gj, int nj, int N, int npairs, bool fp32,
                        hipStream_t st) {
  const size_t n1 = N - 1;
  const size_t n = (size_t)weight_row(N) * n1 * npairs;
  const int g = grid_for(n, 256) < 4096 ? grid_for(n, 256) : 4096;
  if (fp32)
    hipLaunchKernelGGL(k_table<float>, dim3(g), dim3(256), 0, st, (float*)V, pd, gj, nj, N, npairs);
  else
    hipLaunchKernelGGL(k_table<double>, dim3(g), dim3(256), 0, st, (double*)V, pd, gj, nj, N, npairs);
  return hipGetLastError();
}

hipError_t launch_wgen(void* Vc, const double* coef, const double* pdv, const int* terms, int mt, int N, int Mh,
                       int nreal, int j0, int nj, int ncoef, bool fp32, hipStream_t st) {
  if (mt < 8 || mt > 80 || (mt & 7)) return hipErrorInvalidValue;
  const int n1 = N - 1, per = weight_row(N) * n1;
  const int bx = (per + 255) / 256;
  // about 2048 workgroups, each over at least 16 pairs
  const int by = std::max(1, std::min((2048 + bx - 1) / bx, nj / 16));
  const dim3 grid(bx, by);
  if (fp32)
    hipLaunchKernelGGL((k_wgen<float, 4>), grid, dim3(256), 0, st, (float*)Vc, coef, (const double4*)pdv, terms,
                       mt, N, Mh, nreal, j0, nj, ncoef);
  else
    hipLaunchKernelGGL((k_wgen<double, 4>), grid, dim3(256), 0, st, (double*)Vc, coef, (const double4*)pdv, terms,
                       mt, N, Mh, nreal, j0, nj, ncoef);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, double v, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}
hipError_t launch_axpy(double* out, const double* x, double a, const double* y, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(2 * n, 256)), dim3(256), 0, st, out, x, a, y, 2 * n);
  return hipGetLastError();
}
hipError_t launch_heun(double* f, const double* q1, const double* q2, double hh, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_heun, dim3(grid_for(2 * n, 256)), dim3(256), 0, st, f, q1, q2, hh, 2 * n);
  return hipGetLastError();
}
hipError_t launch_fill_int(int* p, int v, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(grid_for((size_t)n, 64)), dim3(64), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_finite(const double* x, size_t n, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_finite, dim3(grid_for(n, 256)), dim3(256), 0, st, x, n, flag);
  return hipGetLastError();
}
hipError_t launch_moments(const double* f, const double* q, double fmin, double L, int N, double* part,
                          int nblocks, hipStream_t st) {
  hipLaunchKernelGGL(k_moments, dim3(nblocks), dim3(256), 0, st, f, q, fmin, L, N, part);
  return hipGetLastError();
}

}  // namespace bzq
