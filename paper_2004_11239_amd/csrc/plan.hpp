// Internal structures shared by the C ABI (capi.cpp), the batched executor
// (batch.cpp) and the request server (server.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/bzq.h"
#include "kernels.hpp"

namespace bzq {

bzq_status fail(bzq_status s, const std::string& msg);

#define BZQ_HIP_TRY(expr)                                                                        \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return ::bzq::fail(BZQ_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

// Device allocations owned by one object, released together.
struct DeviceArena {
  std::vector<void*> allocs;
  size_t bytes = 0;
  ~DeviceArena();
  bzq_status alloc(void** out, size_t nbytes);
  template <typename Tp>
  bzq_status get(Tp** out, size_t nbytes) {
    void* p = nullptr;
    bzq_status s = alloc(&p, nbytes);
    *out = (Tp*)p;
    return s;
  }
};

struct Plan;

// Scratch of the evaluation pipeline for up to `cells` cells per launch.  A
// plan's tables are read-only; every stream that evaluates concurrently needs
// its own workspace.
struct Workspace {
  const Plan* plan = nullptr;
  int cells = 0;
  // chunk geometry of the pipeline on this scratch: pair-twos per chunk, the
  // last stage's splits, pair-twos per block of generated weights; 0 = the
  // plan's G, S, Gw (workspaces made by workspace_init)
  int G = 0, S = 0, Gw = 0;
  bool untimed = false;      // never record timing events (no allocation at all)
  CellStrides cs{};
  void* fc = nullptr;        // cells x (N-1)^3 complex, compute precision
  void* fgrid = nullptr;     // cells x P^3 real
  void* A = nullptr;         // cells x G x P x a_plane(N) complex
  void* B = nullptr;         // cells x G x P x 2 nhp complex
  void* C = nullptr;         // cells x G x P x (N-1) x P complex: plane rows (P = 192 only)
  double* Qpart = nullptr;   // cells x S x nh x n1 complex128
  double* q1 = nullptr;      // cells x N^3 complex128 (Heun stages)
  double* q2 = nullptr;
  double* fs = nullptr;
  void* Vc = nullptr;        // weights of one chunk's pairs (plans with weights on the fly)
  int* flag = nullptr;       // NaN/Inf flag of the input check (a0)
  DeviceArena arena;
};

struct Plan {
  int N = 0, P = 0, n1 = 0, nn = 0, nh = 0, nhp = 0;
  double L = 0, R = 0, gamma = 0, bc = 0, bs = 0, br = 0;
  int N_rho = 0, M = 0, nj = 0;
  // angular kernel: 0 = c t^{-1-s} (1-t)^{-r}; 1 = the Debye-Yukawa kernel of
  // Section 5.6, zero below theta_cut (then bc = 1/4 so that 4 pi bc = pi)
  int kind = 0;
  double theta_cut = 0.0;
  bool fp32 = false;
  int npairs = 0;   // antipodal pairs incl. a zero pad to an even count
  int npt = 0;      // pairs of pairs (packed into one complex transform)
  int G = 0;        // pair-twos per chunk
  int S = 0;        // accumulation splits of the last stage
  int S_cap = 0;    // largest S of any schedule (sizes the accumulators)
  // schedule: kernel variant per stage {z-inverse, plane, z-forward} (0 =
  // default, see stage_variants) and the z-forward workgroups aimed at
  int var[3] = {0, 0, 0};
  int s_target = 1024;
  // compute units of the plan's device and the z-forward workgroups one of
  // them holds, per kernel variant (0: unknown)
  int cus = 0;
  int zfwd_bpc[3] = {0, 0, 0};
  size_t esz = 0;   // bytes per real element (4 or 8)
  std::vector<double> pair_host;  // [npairs][6] for introspection
  // weights on the fly: no table V; per chunk, k_wgen evaluates the series
  // of the angular weight (funk_hecke.hpp) into the workspace
  bool otf = false;
  int mt = 0;                   // coefficient slots per (radial node, |k|^2): multiple of 8, <= 80
  int Gw = 0;                   // pair-twos per block of generated weights
  int Mh = 0;                   // pairs per radial node
  int nreal = 0;                // pairs before the zero-weight pad
  int ncoef = 0;                // |k|^2 values, 0 .. 3 (N/2-1)^2
  double* coef = nullptr;       // [N_rho][ncoef][mt]
  double* pdv = nullptr;        // [npairs][4] sigma, 2 w_sigma / P^3
  int* terms = nullptr;         // [N_rho] terms used per radial node
  // tables (read-only after creation).  Everything but cp is independent of
  // gamma and lives in `shared`, which plans derived for other gammas
  // (derive_plan) hold too; cp lives in the plan's own `tables`.
  void* V = nullptr;            // [npairs][n1][nh] real weights (table plans)
  double* ph = nullptr;         // [npairs][3][2N-3] complex128 phases
  double* cp = nullptr;         // [npairs] w_rho rho^{2+gamma}
  void* tw_pad = nullptr;       // P twiddles (LDS kernels), compute precision
  double* tw_grid = nullptr;    // N twiddles, FP64
  std::shared_ptr<DeviceArena> shared = std::make_shared<DeviceArena>();
  DeviceArena tables;
  // the plan's own workspace (one cell) and FP64 physical-grid scratch
  Workspace ws;
  double* gfc = nullptr;
  double* gA = nullptr;
  double* gC = nullptr;   // plane rows of the physical grid (N = 128 only)
  double* gf = nullptr;
  double* gq = nullptr;
  double* part = nullptr;
  int* flag = nullptr;
  DeviceArena grid_scratch;
  // optional per-launch timing
  int timing = 0;   // bit s set: bracket the launches of stage s with events
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_stage;
  size_t ev_used = 0;
  ~Plan();
  size_t workspace_bytes_per_cell() const;
};

// Grid sizes with an FFT schedule (8, 16, 24, 32, 48, 64, 128)
bool supported_N(int N);
bzq_status workspace_init(Workspace& w, const Plan& p, int cells);
// elements of the plane-row buffer for G pair-twos (0 where the plane fits LDS)
inline size_t plane_rows_elems(const Plan& p, int G) {
  return needs_plane_rows(p.P) ? (size_t)G * p.P * p.n1 * p.P : 0;
}
int effective_variant(const Plan& p, int stage);
// Autotuning cache: "key|value" lines in $BZQ_TUNE_CACHE or ~/.cache/bzq_autotune.txt
std::map<std::string, int> tune_cache_read();
void tune_cache_write(const std::map<std::string, int>& m);
void set_chunking(Plan& p);
// Splits of the last stage for a chunk of G pair-twos under kernel variant zv
// and workgroup target s_target.
int zfwd_splits_for(const Plan& p, int G, int zv, int s_target);
size_t plan_footprint(int N, int N_rho, int M, int precision);
bzq_status create_plan(bzq_plan* out, int N, double L, double R, double gamma, double bc, double bs,
                       double br, int nj, int N_rho, int M, int precision, void* stream, bool otf = false,
                       int kind = 0, double theta_cut = 0.0);
// A plan for another gamma that shares base's gamma-independent tables (the
// weights, phases and twiddles); only its c_p table and scratch are new.
bzq_status derive_plan(const Plan& base, double gamma, bzq_plan* out, hipStream_t st);
// Device bytes of the gamma-independent tables of a plan geometry.
size_t plan_shared_bytes_estimate(int N, int N_rho, int M, int precision);
double power_kernel_constant(double s);
// (c, s, r) of b = c t^{-1-s} (1-t)^{-r} for a bzq_kernel selector (general:
// whether BZQ_KERNEL_GENERAL with the explicit c, s, r is accepted)
bzq_status kernel_params(int kernel, double s, double c, double r, bool general, double* bc, double* bs,
                         double* br);
// bytes of one complex128 N^3 spectral array
inline size_t state_bytes(int N) { return (size_t)N * N * N * 16; }

// Enqueue Q = Q(f) for `cells` cells sharing plan p, using workspace w.
// With upd, the finalize launch also applies that time-step update.  With
// check, the input is checked for NaN/Inf in the ingest launch and the host
// waits for the result (a stream synchronisation) before enqueuing anything
// else: BZQ_ENONFINITE then leaves every output untouched.
bzq_status enqueue_collision(Plan& p, Workspace& w, const PtrPack& f, const PtrPack& Q, int cells,
                             hipStream_t st, const FinUpdate& upd = FinUpdate{}, bool check = false);
// Enqueue n_steps Heun steps in place for `cells` cells (check: of the input
// state, as for enqueue_collision).
bzq_status enqueue_step(Plan& p, Workspace& w, const PtrPack& f, int cells, double dt, int n_steps,
                        hipStream_t st, bool check = false);

// Enqueue n_steps classical Runge-Kutta (RK4) steps in place for `cells` cells.
bzq_status enqueue_step_rk4(Plan& p, Workspace& w, const PtrPack& f, int cells, double dt, int n_steps,
                            hipStream_t st, bool check = false);

// True when the byte ranges [a, a + n) and [b, b + n) overlap.
inline bool ranges_overlap(const void* a, const void* b, size_t n) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + n && y < x + n;
}

inline PtrPack single(const double* p) {
  PtrPack pk{};
  pk.p[0] = const_cast<double*>(p);
  return pk;
}

}  // namespace bzq

struct bzq_plan_s : bzq::Plan {};
