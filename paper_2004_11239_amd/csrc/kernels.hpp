// Launch wrappers for the device kernels of the collision operator.
// Each wrapper dispatches on the padded FFT length P and the precision, and
// enqueues on `stream`; none of them synchronises.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace bzq {

enum ZinvMode { ZINV_PAIRS = 0, ZINV_PLAIN = 1, ZINV_GRID_SIGN = 2 };
enum PlaneMode { PLANE_PRODUCT = 0, PLANE_TO_GRID = 1 };

struct Geometry {
  int N;       // modes per axis incl. the (zero) Nyquist plane
  int P;       // FFT length per axis (3N/2, or N for the physical grid)
};

// Independent cells of one launch (blockIdx.z, or blockIdx.y for the
// element-wise kernels): element strides between consecutive cells' buffers.
struct CellStrides {
  size_t fc;   // compact spectrum
  size_t fg;   // f on the padded grid (or the physical grid)
  size_t a;    // first intermediate
  size_t b;    // second intermediate
  size_t qp;   // partial accumulators (complex128)
  size_t pc;   // plane rows between the passes of the three-pass plane (P = 128, 192)
  int cells;
};

// Row length of the weight table V[pair][i3][c]: the nh = ((N-1)^2 + 1) / 2
// half-spectrum modes of one height, padded to a multiple of 32 entries so
// that every row starts on a 128-byte line and the last stage's tiles (32
// FP32 or 16 FP64 pencils) read whole lines.  The padding entries hold the
// weights of the next modes c >= nh (valid modes, never read).
__host__ __device__ constexpr int weight_row(int N) { return ((((N - 1) * (N - 1) + 1) / 2) + 31) / 32 * 32; }

// Pitch of one height z of the first intermediate A[pair-two][z][c] (and of
// the physical-grid path's A[z][c]): the (N-1)^2 modes of a plane rounded up
// to 16 complex values, so that every plane starts on a 128-byte line.  With
// the unpadded pitch every wave of the axis-3 stage writes lines it covers
// only in part; the entries c >= (N-1)^2 are never written or read.
__host__ __device__ constexpr int a_plane(int N) { return ((N - 1) * (N - 1) + 15) / 16 * 16; }

// Launch shapes aware of the eight XCDs, each with its own L2: workgroups go
// to the XCDs in turn by linear id.
//
// Pencil blocks along the grid's x axis for the z-inverse kernels: rounded up
// to a multiple of 8 when that adds at most an eighth, so that linear id mod
// 8 (the XCD) is the block index mod 8 for every pair-two and each XCD reads
// one eighth of the compact spectrum, which then stays in its L2 (64^3:
// 63 -> 64 blocks of 64 pencils, 128^3: 1009 -> 1016 blocks of 16; the
// padding blocks have no pencils and exit).
__host__ __device__ constexpr int xcd_pencil_blocks(int gx) {
  return ((gx + 7) / 8 * 8) - gx <= gx / 8 ? (gx + 7) / 8 * 8 : gx;
}

// Tile of workgroup x (of gx along the grid's x axis) when LG consecutive
// tiles share the 128-byte lines of their rows: the workgroups
// x = q 8 LG + k + 8 j (j < LG) all run on one XCD at nearly the same time
// and take the tiles q 8 LG + k LG + j, the LG tiles of one line.  Within a
// whole group of 8 LG workgroups this is a bijection (an LG x 8 transpose); a
// ragged last group keeps the identity map.
template <int LG>
__host__ __device__ constexpr int xcd_line_tile(int x, int gx) {
  return (LG == 1 || (x / (8 * LG) + 1) * 8 * LG > gx)
             ? x
             : x / (8 * LG) * 8 * LG + LG * ((x % (8 * LG)) & 7) + ((x % (8 * LG)) >> 3);
}

// Per-cell device pointers passed by value (at most kMaxCells per launch).
constexpr int kMaxCells = 64;
struct PtrPack {
  double* p[kMaxCells];
};

// Compact spectral copy: fc[i1][i2][i3] (centred, (N-1)^3) from the FFT-order
// complex128 array f (N^3).  fp32 selects the element type of fc.  With flag
// != nullptr, flag[0] is set to 1 if any value read is NaN or Inf (it is
// never cleared here).
hipError_t launch_ingest(const PtrPack& f, void* fc, size_t fc_stride, int cells, int N, bool fp32,
                         hipStream_t st, int* flag = nullptr);

// launch_ingest and launch_zinv(mode ZINV_PLAIN, one pair-two) in one launch,
// for the lengths whose pencil fits the register file (zinv_ingest_fits):
// fc as launch_ingest writes it, A[pair-two 0] as launch_zinv writes it.
bool zinv_ingest_fits(int P, bool fp32);

// The two-dimensional operator's pipeline at N = 64 (P = 96) with register FFTs
// (one workgroup of 256 threads per pair-two loop s, s + S, ...): fc and fgrid
// as the 2-D prep writes them, V the 2-D weight table, ph the 2-D phases,
// Qpart[S][nh] the partial sums (written).
hipError_t launch_collide2d_reg(const void* fc, const void* fgrid, const void* V, const double* ph, const double* cp,
                                double* Qpart, int N, int npt, int S, bool fp32, hipStream_t st);
hipError_t launch_zinv_ingest(const PtrPack& f, void* fc, void* A, Geometry g, bool fp32, const CellStrides& cs,
                              hipStream_t st, int* flag = nullptr);

// Step 1 of the pipeline: modulate (mode ZINV_PAIRS) and inverse-transform along
// axis 3; writes A[pt][z][c] for pt < npt, z < P, c < (N-1)^2.
hipError_t launch_zinv(const void* fc, const double* phase, void* A, const void* tw, Geometry g,
                       int pair0, int npt, int mode, bool fp32, const CellStrides& cs, hipStream_t st,
                       int variant = 0);

// Step 2: per (pt, z) plane: inverse along axes 2 and 1, product with the
// physical f (mode PLANE_PRODUCT) or output of the real grid (PLANE_TO_GRID),
// forward along axes 1 and 2.  At P = 128 and 192 a plane does not fit LDS
// and the stage runs in three passes through C (needs_plane_rows): C holds,
// per pair-two and z plane, the N-1 mode rows of P values (npt x P x (N-1) x P
// complex, cell stride cs.pc); elsewhere C is unused.
bool needs_plane_rows(int P);
hipError_t launch_plane(const void* A, void* B, const void* fgrid, void* gridout, const void* tw,
                        Geometry g, int npt, int mode, bool fp32, const CellStrides& cs, hipStream_t st,
                        int variant = 0, void* C = nullptr);

// Step 3: forward along axis 3, split the two packed pairs, apply the stored
// weights and the phase e^{i a k.sigma}, accumulate in FP64 into Qpart[s].
// The weight of pair j is row j - vpair0 of V (0 for a plan-wide table, the
// chunk's first pair for weights generated per chunk).  With first = true the
// launch writes every partial Qpart[s < S] instead of adding to it (the first
// launch of an evaluation, so that no clearing pass is needed).
hipError_t launch_zfwd(const void* B, const void* V, const double* phase, const double* cp,
                       double* Qpart, const void* tw, Geometry g, int pair0, int npt, int S,
                       bool fp32, const CellStrides& cs, hipStream_t st, int variant = 0, int vpair0 = 0,
                       bool first = false);

// Workgroups of the z-forward kernel of `variant` (0 = default) that one
// compute unit holds at once on the current device (0 if the query fails).
int zfwd_blocks_per_cu(int P, bool fp32, int variant);

// Weights of pairs j0 .. j0+nj-1 into Vc[j - j0][n1][nh] (compute precision)
// from the series of the angular weight in Chebyshev form:
// Re(e^{-ix} F) = sum_k coef[p][n][k] T_k(2 t^2 - 1), t = k.sigma/|k|, for
// radial node p and n = |k|^2 < ncoef (k < terms[p], zero above);
// pdv[j] = {sigma_x, sigma_y, sigma_z, 2 w_sigma / P^3} (0 for the padding
// pair).  mt (coefficient slots) is a multiple of 8, at most 80, and at
// least every terms[p] rounded up to a multiple of 8.
hipError_t launch_wgen(void* Vc, const double* coef, const double* pdv, const int* terms, int mt, int N, int Mh,
                       int nreal, int j0, int nj, int ncoef, bool fp32, hipStream_t st);

// Kernel variants of the stages {0 z-inverse, 1 plane, 2 z-forward}: bit v of
// stage_variants is set when variant v runs for padded length P (1 = one whole
// pencil per lane, 2 = two waves per pencil / pipelined z-forward);
// stage_default_variant is the one variant 0 selects.
unsigned stage_variants(int stage, int P, bool fp32);
int stage_default_variant(int stage, int P, bool fp32);

// A time-step update fused into the finalize launch, applied at every element
// the launch writes of Q (N^3 complex128 per cell, cell c of a workspace buffer
// at ws + c * wstride doubles; f is the state):
//   FIN_STAGE: ws = f + a Q       (ws: the intermediate state)
//   FIN_HEUN:  f  = f + a (ws + Q) (ws: the first stage's Q)
// the same arithmetic as launch_axpy_cells / launch_heun_cells.
enum FinUpdateMode { FIN_NONE = 0, FIN_STAGE = 1, FIN_HEUN = 2 };
struct FinUpdate {
  int mode = FIN_NONE;
  double a = 0.0;
  double* ws = nullptr;
  size_t wstride = 0;
  PtrPack f{};
};

// Sum of the S partial accumulators and Hermitian completion into Q (N^3 FFT
// order), with an optional fused update (FinUpdate).
hipError_t launch_finalize(const double* Qpart, const PtrPack& Q, size_t qp_stride, int cells, int N, int S,
                           hipStream_t st, const FinUpdate& upd = FinUpdate{});
// per cell: out = x + a y and f += h (q1 + q2)  (n complex128 each)
hipError_t launch_axpy_cells(const PtrPack& out, const PtrPack& x, double a, const PtrPack& y, size_t n,
                             int cells, hipStream_t st);
hipError_t launch_heun_cells(const PtrPack& f, const PtrPack& q1, const PtrPack& q2, double hh, size_t n,
                             int cells, hipStream_t st);

// Real weight table V[pair][c][i3] (FP64 arithmetic, stored as float or double).
hipError_t launch_table(void* V, const double* pairdat, const double* gj, int nj, int N,
                        int npairs, bool fp32, hipStream_t st);

// Mixed-size launches (FP32 bulk, N in {16, 24, 32}): one launch per pipeline
// stage over the cells of a round, one work item (cell, workgroup of that
// cell's stage) per workgroup, from a device work table (offs: first item of
// each cell).  Stages, in order: the compact copy of f with its transform
// along axis 3, f on the padded grid, the z-inverse, the plane, the z-forward
// with the weights, the finalisation.
enum MixStage { MIX_INGEST = 0, MIX_GRID = 1, MIX_ZINV = 2, MIX_PLANE = 3, MIX_ZFWD = 4, MIX_FINAL = 5, MIX_STAGES = 6 };
struct MixCell {
  int N;               // 16, 24 or 32
  int npt, S;          // pair-twos (one chunk), splits of the last stage
  int cell;            // index of the cell in its batch (output of a plain evaluation)
  double2* f;          // state: the input of a plain evaluation and of the first Heun stage
  double2* fs;         // stage state (input of the second Heun stage)
  double2* q1;         // Q of the first Heun stage
  double2* q2;         // Q of the second
  void* fc;            // workspace of the cell's slot (complex FP32, FP32, complex FP32 x 2)
  float* fgrid;
  void* A;
  void* B;
  double2* Qpart;
  const float* V;      // tables of the cell's plan
  const double2* ph;
  const double* cp;
};
// Whether a plan (N, precision, kernel variants as used) runs in the mixed
// launches, and the work items of stage `stage` of one such cell.
bool mix_supported(int N, bool fp32, int zinv_variant, int plane_variant, int zfwd_variant);
int mix_items(int stage, int N, int npt, int S);
// phase 0: Q = Q(f) into outs[cell]; 1: q1 = Q(f), fs = f + a q1; 2: q2 = Q(fs),
// f += a (q1 + q2) (the two evaluations of a Heun step with a = dt, dt/2)
hipError_t launch_mix(int stage, const MixCell* cells, const int* offs, int ncells, int total, int phase, double a,
                      double2* const* outs, hipStream_t st);

// Size of the static device scratch of bzq_collision_noalloc, and its device
// address on the current device (looked up once per device, then cached).
constexpr size_t kNoAllocScratchBytes = 128ull << 20;
hipError_t noalloc_scratch(void** out);

hipError_t launch_fill(double* p, double v, size_t n, hipStream_t st);
hipError_t launch_fill_int(int* p, int v, int n, hipStream_t st);
// out = x + a y  (n complex128)
hipError_t launch_axpy(double* out, const double* x, double a, const double* y, size_t n,
                       hipStream_t st);
// f += h (q1 + q2)
hipError_t launch_heun(double* f, const double* q1, const double* q2, double h, size_t n,
                       hipStream_t st);
// flag[0] = 1 if any of the n doubles is not finite (flag must be zeroed first)
hipError_t launch_finite(const double* x, size_t n, int* flag, hipStream_t st);
// per-block partial sums over the N^3 grid (layout [z][x][y]):
//   part[b*8 + {0..4}] = sum f, f v1, f v2, f v3, f |v|^2;  part[b*8+5] = max f
//   when q != nullptr and fmin >= 0: part[b*8+6] = sum q ln f over f > fmin
hipError_t launch_moments(const double* f, const double* q, double fmin, double L, int N,
                          double* part, int nblocks, hipStream_t st);

}  // namespace bzq
