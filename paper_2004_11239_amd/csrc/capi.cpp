// The C ABI of include/bzq.h: plan construction (quadrature rules, weight
// tables), workspaces, and the host-side orchestration of the device pipeline
// for single cells.  Batched cells live in batch.cpp, the request server in
// server.cpp.
//
// A plan holds, for the operator of eq. realQ:
//   * the antipodal quadrature pairs (rho_p, sigma_q+), sigma_q+ from the half
//     of the Lebedev rule with a positive leading coordinate; the pair stands
//     for sigma and -sigma together, which is exact because the rule is
//     centrally symmetric with equal weights (F(k, rho, -sigma) is the complex
//     conjugate of F(k, rho, sigma) and the two convolutions differ by the
//     phase e^{i pi rho k.sigma / L});
//   * the real weight V_j(k) = 2 w_sigma Re(e^{-ix} F(k, rho, sigma)) / P^3,
//     x = pi rho k.sigma / (2L), on the half spectrum, built on the device;
//     Phi(rho) rho^2 w_rho = w_rho rho^{2+gamma} is applied per pair at run
//     time;
//   * the separable phase tables e^{i pi rho n sigma_d / (2L)} for |n| <= N-2;
//   * twiddles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "funk_hecke.hpp"
#include "plan.hpp"
#include "quadrature.hpp"

namespace bzq {

namespace {
thread_local std::string g_last_error;
const long double kPi = 3.141592653589793238462643383279502884L;
constexpr int kMomentBlocks = 256;

}  // namespace

bool supported_N(int N) { return N == 8 || N == 16 || N == 24 || N == 32 || N == 48 || N == 64 || N == 128; }

bzq_status fail(bzq_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

DeviceArena::~DeviceArena() {
  for (void* p : allocs) (void)hipFree(p);
}

bzq_status DeviceArena::alloc(void** out, size_t nbytes) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, nbytes ? nbytes : 16);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return fail(BZQ_ENOMEM, "hipMalloc(" + std::to_string(nbytes) + ") failed: " + hipGetErrorString(e));
  }
  allocs.push_back(p);
  bytes += nbytes;
  *out = p;
  return BZQ_OK;
}

Plan::~Plan() {
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
}

size_t Plan::workspace_bytes_per_cell() const {
  const size_t N3 = (size_t)N * N * N;
  return (size_t)n1 * nn * 2 * esz + (size_t)P * P * P * esz + (size_t)G * P * a_plane(N) * 2 * esz +
         (size_t)G * P * 2 * nhp * 2 * esz + plane_rows_elems(*this, G) * 2 * esz + (size_t)S_cap * nh * n1 * 16 +
         3 * N3 * 16 +
         (otf ? (size_t)2 * Gw * weight_row(N) * n1 * esz : 0) + 4 * sizeof(int);
}

bzq_status workspace_init(Workspace& w, const Plan& p, int cells) {
  if (cells < 1 || cells > kMaxCells) return fail(BZQ_EINVAL, "cells per launch must lie in [1, 64]");
  w.plan = &p;
  w.cells = cells;
  w.G = w.S = w.Gw = 0;   // the plan's geometry, whatever its schedule
  w.cs.fc = (size_t)p.n1 * p.nn;
  w.cs.fg = (size_t)p.P * p.P * p.P;
  w.cs.a = (size_t)p.G * p.P * a_plane(p.N);
  w.cs.b = (size_t)p.G * p.P * 2 * p.nhp;
  w.cs.qp = (size_t)p.S_cap * p.nh * p.n1;
  w.cs.pc = plane_rows_elems(p, p.G);
  w.cs.cells = cells;
  const size_t N3 = (size_t)p.N * p.N * p.N;
  bzq_status s;
  if ((s = w.arena.get(&w.fc, cells * w.cs.fc * 2 * p.esz)) != BZQ_OK) return s;
  if ((s = w.arena.get(&w.fgrid, cells * w.cs.fg * p.esz)) != BZQ_OK) return s;
  if ((s = w.arena.get(&w.A, cells * w.cs.a * 2 * p.esz)) != BZQ_OK) return s;
  if ((s = w.arena.get(&w.B, cells * w.cs.b * 2 * p.esz)) != BZQ_OK) return s;
  if (w.cs.pc && (s = w.arena.get(&w.C, cells * w.cs.pc * 2 * p.esz)) != BZQ_OK) return s;
  if ((s = w.arena.get(&w.Qpart, cells * w.cs.qp * 16)) != BZQ_OK) return s;
  if ((s = w.arena.get(&w.q1, cells * N3 * 16)) != BZQ_OK) return s;
  if ((s = w.arena.get(&w.q2, cells * N3 * 16)) != BZQ_OK) return s;
  if ((s = w.arena.get(&w.fs, cells * N3 * 16)) != BZQ_OK) return s;
  if (p.otf && (s = w.arena.get(&w.Vc, (size_t)2 * p.Gw * weight_row(p.N) * p.n1 * p.esz)) != BZQ_OK) return s;
  if ((s = w.arena.get(&w.flag, 4 * sizeof(int))) != BZQ_OK) return s;
  return BZQ_OK;
}

namespace {
std::string tune_path() {
  const char* e = std::getenv("BZQ_TUNE_CACHE");
  if (e && *e) return e;
  const char* h = std::getenv("HOME");
  return std::string(h && *h ? h : "/tmp") + "/.cache/bzq_autotune.txt";
}
}  // namespace

std::map<std::string, int> tune_cache_read() {
  std::map<std::string, int> m;
  std::ifstream in(tune_path());
  std::string line;
  while (std::getline(in, line)) {
    const size_t bar = line.rfind('|');
    if (bar == std::string::npos) continue;
    m[line.substr(0, bar)] = std::atoi(line.c_str() + bar + 1);
  }
  return m;
}

void tune_cache_write(const std::map<std::string, int>& m) {
  const std::string path = tune_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) (void)::mkdir(path.substr(0, slash).c_str(), 0755);
  std::ofstream out(path, std::ios::trunc);
  if (!out) return;   // a read-only home only loses the cache
  for (const auto& kv : m) out << kv.first << "|" << kv.second << "\n";
}

int effective_variant(const Plan& p, int stage) {
  return p.var[stage] ? p.var[stage] : stage_default_variant(stage, p.P, p.fp32);
}

// z-forward workgroup targets a schedule can choose
constexpr int kSTargets[3] = {512, 1024, 2048};

// Splits of the z-forward stage for kernel variant zv: about s_target
// workgroups of tq pencils, at most one per group of pair-twos.  Pipelined
// kernel: 32 pencils, one pair-two per step; other register kernels: 32 or 16
// pencils, 2 or 4 pair-twos per step; LDS kernels (FP64 P > 48, FP32 P > 96):
// 8 pencils.
// When the kernel's residency is known and at most s_target, the workgroups
// fill whole rounds of the chip: s_target is rounded down to a multiple of the
// resident workgroups and S down to what fits it, so that no launch ends with
// a nearly empty round (64^3 FP32: 1008 workgroups on 512 slots instead of
// 1071).  S never exceeds its value without the rounding.
int zfwd_splits_for(const Plan& p, int G, int zv, int s_target) {
  const bool pipe = zv == 2 && (stage_variants(2, p.P, p.fp32) & 0x4u);
  const bool reg_zfwd = p.fp32 ? p.P <= 96 : p.P <= 48;
  const int tq = pipe ? 32 : reg_zfwd ? (p.fp32 ? 32 : 16) : 8;
  const int pt_group = pipe ? 1 : reg_zfwd ? (p.fp32 ? 2 : 4) : 1;
  const int groups = (G + pt_group - 1) / pt_group;
  const int tiles = (p.nh + tq - 1) / tq;
  const int slots = p.cus * (zv >= 1 && zv <= 2 ? p.zfwd_bpc[zv] : 0);
  if (slots > 0 && slots <= s_target) return std::max(1, std::min(groups, s_target / slots * slots / tiles));
  return std::max(1, std::min(groups, (s_target + tiles - 1) / tiles));
}
int zfwd_splits(const Plan& p, int zv, int s_target) { return zfwd_splits_for(p, p.G, zv, s_target); }

// Chunking of the pair loop: the pipeline intermediates stay below 2 GiB per
// cell (BZQ_CHUNK_MB; one chunk per evaluation up to N = 32 in both
// precisions).  Fewer, larger chunks mean fewer launches and fewer round trips
// of the last stage's partial sums: at 64^3 1024 / 2048 / 4096 MiB took
// 19.32 / 19.02 / 19.00 ms per FP32 evaluation, 42.85 / 41.44 / 40.65 ms per
// FP64 one.  The splits S of the last
// stage give about s_target workgroups (enough to fill the chip) but no more
// than there are groups of pair-twos.  S_cap bounds S over every schedule.
void set_chunking(Plan& p) {
  p.esz = p.fp32 ? 4 : 8;
  p.nhp = (p.nh + 15) / 16 * 16;
  const size_t per_pt = ((size_t)p.P * (a_plane(p.N) + 2 * p.nhp) + plane_rows_elems(p, 1)) * 2 * p.esz;
  const char* env = std::getenv("BZQ_CHUNK_MB");
  const size_t cap = (env && std::atoll(env) > 0 ? (size_t)std::atoll(env) : 2048ull) << 20;
  p.G = (int)std::max<size_t>(1, std::min<size_t>((size_t)p.npt, cap / per_pt));
  // weights on the fly: pair-twos per generated block of weights (below
  // BZQ_OTF_MB, default 256 MiB: at 64^3 FP32 blocks of 32 / 64 / 128 MiB took
  // 27.9 / 24.8 / 23.8 ms per evaluation, 192 MiB and more 22.9 ms, since every
  // block is one more last-stage launch over fewer pair-twos), and at most half
  // of the pair-twos, so that a plan with weights on the fly never holds as
  // many weight bytes as the table it replaces (at 32^3 one block would hold
  // all of them)
  const char* envw = std::getenv("BZQ_OTF_MB");
  const size_t capw = (envw && std::atoll(envw) > 0 ? (size_t)std::atoll(envw) : 256ull) << 20;
  const size_t per_w = (size_t)2 * weight_row(p.N) * p.n1 * p.esz;
  const size_t half = ((size_t)p.npt + 1) / 2;
  p.Gw = p.otf ? (int)std::max<size_t>(1, std::min<size_t>(std::min<size_t>((size_t)p.G, capw / per_w), half)) : 0;
  p.S = zfwd_splits(p, effective_variant(p, 2), p.s_target);
  p.S_cap = p.S;
  for (int v = 1; v <= 2; ++v)
    if (stage_variants(2, p.P, p.fp32) >> v & 1)
      for (int t : kSTargets) p.S_cap = std::max(p.S_cap, zfwd_splits(p, v, t));
}

// Device bytes a plan will hold (tables, its workspace, grid scratch), from
// its geometry alone; Lebedev rules are centrally symmetric, so the number of
// antipodal pairs is N_rho M / 2 rounded up to even.
size_t plan_footprint(int N, int N_rho, int M, int precision) {
  Plan p;
  p.N = N;
  p.P = 3 * N / 2;
  p.n1 = N - 1;
  p.nn = p.n1 * p.n1;
  p.nh = (p.nn + 1) / 2;
  p.fp32 = precision == BZQ_FP32_ACC64;
  const int nreal = N_rho * (M / 2);
  p.npairs = nreal + (nreal & 1);
  p.npt = p.npairs / 2;
  set_chunking(p);
  const size_t n3 = (size_t)N * N * N;
  const size_t tables = plan_shared_bytes_estimate(N, N_rho, M, precision) + (size_t)p.npairs * 8;
  const size_t grid = (size_t)p.n1 * p.nn * 16 + (size_t)N * p.nn * 16 + 2 * n3 * 8 + 256 * 8 * 8 + 16 +
                      (needs_plane_rows(N) ? (size_t)N * p.n1 * N * 16 : 0);
  return tables + p.workspace_bytes_per_cell() + grid;
}

namespace {
bzq_status alloc_scratch(Plan* p);
}  // namespace

size_t plan_shared_bytes_estimate(int N, int N_rho, int M, int precision) {
  const int P = 3 * N / 2, n1 = N - 1;
  const size_t esz = precision == BZQ_FP32_ACC64 ? 4 : 8;
  const int nreal = N_rho * (M / 2);
  const size_t npairs = nreal + (nreal & 1);
  return npairs * weight_row(N) * n1 * esz + npairs * 3 * (2 * N - 3) * 16 + (size_t)P * 2 * esz + (size_t)N * 16;
}

bzq_status derive_plan(const Plan& base, double gamma, bzq_plan* out, hipStream_t st) {
  if (!out) return fail(BZQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (!(gamma > -3.0 && gamma <= 1.0)) return fail(BZQ_EINVAL, "gamma must lie in (-3, 1]");
  bzq_plan_s* p = new bzq_plan_s();
  // geometry, schedule and the shared tables
  p->N = base.N; p->P = base.P; p->n1 = base.n1; p->nn = base.nn; p->nh = base.nh; p->nhp = base.nhp;
  p->L = base.L; p->R = base.R; p->gamma = gamma;
  p->bc = base.bc; p->bs = base.bs; p->br = base.br;
  p->N_rho = base.N_rho; p->M = base.M; p->nj = base.nj; p->fp32 = base.fp32;
  p->kind = base.kind; p->theta_cut = base.theta_cut;
  p->npairs = base.npairs; p->npt = base.npt; p->G = base.G; p->S = base.S; p->S_cap = base.S_cap;
  for (int i = 0; i < 3; ++i) p->var[i] = base.var[i];
  p->s_target = base.s_target; p->esz = base.esz;
  p->cus = base.cus;
  for (int i = 0; i < 3; ++i) p->zfwd_bpc[i] = base.zfwd_bpc[i];
  p->otf = base.otf; p->mt = base.mt; p->Gw = base.Gw; p->Mh = base.Mh; p->nreal = base.nreal;
  p->ncoef = base.ncoef; p->coef = base.coef; p->pdv = base.pdv; p->terms = base.terms;
  p->V = base.V; p->ph = base.ph; p->tw_pad = base.tw_pad; p->tw_grid = base.tw_grid;
  p->shared = base.shared;
  p->pair_host = base.pair_host;
  // c_p = w_rho rho^{2+gamma} for the new gamma
  std::vector<double> rho, wr;
  gauss_legendre(p->N_rho, p->R, rho, wr);
  std::vector<double> cp(p->npairs, 0.0);
  for (int j = 0; j < p->nreal; ++j) {
    const int ip = j / p->Mh;
    cp[j] = (double)((long double)wr[ip] * powl((long double)rho[ip], 2.0L + gamma));
    p->pair_host[6 * j + 5] = cp[j];
  }
  bzq_status s;
  hipError_t e = hipSuccess;
  if ((s = p->tables.get(&p->cp, cp.size() * sizeof(double))) != BZQ_OK || (s = alloc_scratch(p)) != BZQ_OK) {
    delete p;
    return s;
  }
  e = hipMemcpyAsync(p->cp, cp.data(), cp.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete p;
    return fail(BZQ_EDEVICE, std::string("derived plan: ") + hipGetErrorString(e));
  }
  *out = p;
  return BZQ_OK;
}

namespace {

// Tables of a plan whose weights are evaluated on the fly (funk_hecke.hpp):
// the series coefficients per radial node and |k|^2, and the pair
// directions and scales.
bzq_status build_series(Plan* p, const std::vector<double>& rho, int Mh, int nreal, hipStream_t st) {
  const int h = p->N / 2;
  p->Mh = Mh;
  p->nreal = nreal;
  p->ncoef = 3 * (h - 1) * (h - 1) + 1;
  std::vector<int> terms(p->N_rho);
  int need = 1;
  for (int ip = 0; ip < p->N_rho; ++ip) {
    const double a = (double)(kPi * rho[ip] / (2.0L * p->L));
    terms[ip] = fh_lmax(a * std::sqrt((double)(p->ncoef - 1))) / 2 + 1;
    need = std::max(need, terms[ip]);
  }
  if (need > 80)
    return fail(BZQ_EUNSUPPORTED, "weights on the fly: a |k| too large for the series (at most 80 even terms)");
  p->mt = (need + 7) / 8 * 8;   // coefficient slots: the kernel unrolls in multiples of 8 terms
  std::vector<long double> mu, Ml;
  if (!fh_moments(2 * (need - 1), p->bc, p->bs, p->br, mu)) return fail(BZQ_EINVAL, "Gauss-Jacobi rule failed");
  fh_cheb_matrix(need, Ml);
  std::vector<double> M(Ml.begin(), Ml.end());
  // coef[p][n][k]: Chebyshev coefficients in u = 2t^2 - 1 of the series for
  // radial node p and |k|^2 = n
  std::vector<double> coef((size_t)p->N_rho * p->ncoef * p->mt, 0.0);
  std::vector<long double> jl;
  std::vector<double> c(need);
  for (int ip = 0; ip < p->N_rho; ++ip) {
    const long double a = kPi * rho[ip] / (2.0L * p->L);
    const int tp = terms[ip];
    for (int n = 0; n < p->ncoef; ++n) {
      fh_sph_bessel(2 * (tp - 1), a * sqrtl((long double)n), jl);
      for (int m = 0; m < tp; ++m) {
        const int l = 2 * m;
        c[m] = (double)((2 * l + 1) * ((m & 1) ? -1.0L : 1.0L) * mu[m] * jl[l]);
      }
      double* d = &coef[((size_t)ip * p->ncoef + n) * p->mt];
      for (int k = 0; k < tp; ++k) {
        double acc = 0.0;
        for (int m = k; m < tp; ++m) acc += M[(size_t)k * need + m] * c[m];
        d[k] = acc;
      }
    }
  }
  std::vector<double> pdv((size_t)p->npairs * 4, 0.0);
  const long double P3 = (long double)p->P * p->P * p->P;
  for (int j = 0; j < nreal; ++j) {
    const double* ho = &p->pair_host[6 * j];
    pdv[4 * j] = ho[1];
    pdv[4 * j + 1] = ho[2];
    pdv[4 * j + 2] = ho[3];
    pdv[4 * j + 3] = (double)(2.0L * ho[4] / P3);
  }
  bzq_status s;
  if ((s = p->shared->get(&p->coef, coef.size() * sizeof(double))) != BZQ_OK) return s;
  if ((s = p->shared->get(&p->pdv, pdv.size() * sizeof(double))) != BZQ_OK) return s;
  if ((s = p->shared->get(&p->terms, terms.size() * sizeof(int))) != BZQ_OK) return s;
  BZQ_HIP_TRY(hipMemcpyAsync(p->coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, st));
  BZQ_HIP_TRY(hipMemcpyAsync(p->pdv, pdv.data(), pdv.size() * sizeof(double), hipMemcpyHostToDevice, st));
  BZQ_HIP_TRY(hipMemcpyAsync(p->terms, terms.data(), terms.size() * sizeof(int), hipMemcpyHostToDevice, st));
  // the host vectors go out of scope: wait for the copies
  BZQ_HIP_TRY(hipStreamSynchronize(st));
  return BZQ_OK;
}

// The plan's own workspace (one cell) and its FP64 physical-grid scratch.
bzq_status alloc_scratch(Plan* p) {
  const int N = p->N, nn = p->nn;
  bzq_status s;
  if ((s = workspace_init(p->ws, *p, 1)) != BZQ_OK) return s;
  const size_t n3 = (size_t)N * N * N;
  if ((s = p->grid_scratch.get(&p->gfc, (size_t)p->n1 * nn * 2 * sizeof(double))) != BZQ_OK) return s;
  if ((s = p->grid_scratch.get(&p->gA, (size_t)N * a_plane(N) * 2 * sizeof(double))) != BZQ_OK) return s;
  if (needs_plane_rows(N) &&
      (s = p->grid_scratch.get(&p->gC, (size_t)N * p->n1 * N * 2 * sizeof(double))) != BZQ_OK)
    return s;
  if ((s = p->grid_scratch.get(&p->gf, n3 * sizeof(double))) != BZQ_OK) return s;
  if ((s = p->grid_scratch.get(&p->gq, n3 * sizeof(double))) != BZQ_OK) return s;
  if ((s = p->grid_scratch.get(&p->part, (size_t)kMomentBlocks * 8 * sizeof(double))) != BZQ_OK) return s;
  if ((s = p->grid_scratch.get(&p->flag, sizeof(int) * 4)) != BZQ_OK) return s;
  return BZQ_OK;
}

bzq_status build_plan(Plan* p, hipStream_t st) {
  const int N = p->N, P = p->P, nh = p->nh;
  // -- quadrature
  std::vector<double> rho, wr;
  gauss_legendre(p->N_rho, p->R, rho, wr);
  std::vector<double> leb, half;
  if (!lebedev_rule(p->M, leb)) return fail(BZQ_EINVAL, "M is not the size of an available Lebedev rule");
  const int Mh = lebedev_half(leb, half);
  if (Mh < 1) return fail(BZQ_EINVAL, "sphere rule is not centrally symmetric");
  std::vector<double> gt, gw;
  if (p->kind == 1) {
    if (!debye_rule(p->theta_cut, gt, gw)) return fail(BZQ_EINVAL, "theta_cut must lie in [0, pi/3)");
    p->nj = (int)gt.size();
  } else if (!gauss_jacobi01(p->nj, p->bs, p->br, gt, gw)) {
    return fail(BZQ_EINVAL, "Gauss-Jacobi rule failed");
  }
  const int nreal = p->N_rho * Mh;
  p->npairs = nreal + (nreal & 1);
  p->npt = p->npairs / 2;
  p->Mh = Mh;
  p->nreal = nreal;
  // -- per-pair data
  const int PL = 2 * N - 3;
  std::vector<double> pd((size_t)p->npairs * 8, 0.0), cp(p->npairs, 0.0), ph((size_t)p->npairs * 3 * PL * 2);
  p->pair_host.assign((size_t)p->npairs * 6, 0.0);
  const long double P3 = (long double)P * P * P;
  for (int j = 0; j < p->npairs; ++j) {
    long double a = 0, sx = 0, sy = 0, sz = 1, wq = 0, c = 0, r = 0;
    if (j < nreal) {
      const int ip = j / Mh, iq = j % Mh;
      r = rho[ip];
      a = kPi * r / (2.0L * p->L);
      sx = half[4 * iq];
      sy = half[4 * iq + 1];
      sz = half[4 * iq + 2];
      wq = half[4 * iq + 3];
      c = (long double)wr[ip] * powl(r, 2.0L + p->gamma);
    }
    pd[8 * j + 0] = (double)a;
    pd[8 * j + 1] = (double)sx;
    pd[8 * j + 2] = (double)sy;
    pd[8 * j + 3] = (double)sz;
    pd[8 * j + 4] = (double)(2.0L * wq * 4.0L * kPi * p->bc / P3);
    cp[j] = (double)c;
    double* ho = &p->pair_host[6 * j];
    ho[0] = (double)r; ho[1] = (double)sx; ho[2] = (double)sy; ho[3] = (double)sz;
    ho[4] = (double)wq; ho[5] = (double)c;
    const long double sd[3] = {sx, sy, sz};
    for (int d = 0; d < 3; ++d)
      for (int n = -(N - 2); n <= N - 2; ++n) {
        const long double ang = a * sd[d] * n;
        const size_t o = (((size_t)j * 3 + d) * PL + (n + N - 2)) * 2;
        ph[o] = (double)cosl(ang);
        ph[o + 1] = (double)sinl(ang);
      }
  }
  // the default workgroup target of the last stage: 512 at P = 96 (64^3,
  // pipelined z-forward: 3.75 vs 3.92 ms FP32, 8.11 vs 8.54 ms FP64 per
  // evaluation against 1024), 1024 elsewhere (48^3 FP32: 1.14 vs 1.39 ms)
  p->s_target = P == 96 ? 512 : 1024;
  // residency of the z-forward kernels on this device (sizes the splits S)
  {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) {
      for (int v = 1; v <= 2; ++v)
        if (stage_variants(2, p->P, p->fp32) >> v & 1) p->zfwd_bpc[v] = zfwd_blocks_per_cu(p->P, p->fp32, v);
    } else {
      p->cus = 0;
    }
  }
  set_chunking(*p);
  // -- tables
  bzq_status s;
  const size_t vcount = (size_t)p->npairs * weight_row(N) * p->n1;
  if (p->otf) {
    if ((s = build_series(p, rho, Mh, nreal, st)) != BZQ_OK) return s;
  } else if ((s = p->shared->get(&p->V, vcount * p->esz)) != BZQ_OK) {
    return s;
  }
  if ((s = p->shared->get(&p->ph, ph.size() * sizeof(double))) != BZQ_OK) return s;
  if ((s = p->tables.get(&p->cp, cp.size() * sizeof(double))) != BZQ_OK) return s;
  if ((s = p->shared->get(&p->tw_pad, (size_t)P * 2 * p->esz)) != BZQ_OK) return s;
  if ((s = p->shared->get(&p->tw_grid, (size_t)N * 2 * sizeof(double))) != BZQ_OK) return s;
  // -- the plan's own workspace and grid scratch
  if ((s = alloc_scratch(p)) != BZQ_OK) return s;
  DeviceArena tmp;
  double* d_pd = nullptr;
  double* d_gj = nullptr;
  if ((s = tmp.get(&d_pd, pd.size() * sizeof(double))) != BZQ_OK) return s;
  if ((s = tmp.get(&d_gj, 2 * gt.size() * sizeof(double))) != BZQ_OK) return s;
  std::vector<double> gj(gt);
  gj.insert(gj.end(), gw.begin(), gw.end());
  // twiddles e^{-2 pi i m / n}
  std::vector<double> twp(2 * P), twg(2 * N);
  for (int m = 0; m < P; ++m) {
    twp[2 * m] = (double)cosl(2 * kPi * m / P);
    twp[2 * m + 1] = (double)-sinl(2 * kPi * m / P);
  }
  for (int m = 0; m < N; ++m) {
    twg[2 * m] = (double)cosl(2 * kPi * m / N);
    twg[2 * m + 1] = (double)-sinl(2 * kPi * m / N);
  }
  std::vector<float> twpf(twp.begin(), twp.end());
  BZQ_HIP_TRY(hipMemcpyAsync(p->ph, ph.data(), ph.size() * sizeof(double), hipMemcpyHostToDevice, st));
  BZQ_HIP_TRY(hipMemcpyAsync(p->cp, cp.data(), cp.size() * sizeof(double), hipMemcpyHostToDevice, st));
  BZQ_HIP_TRY(hipMemcpyAsync(d_pd, pd.data(), pd.size() * sizeof(double), hipMemcpyHostToDevice, st));
  BZQ_HIP_TRY(hipMemcpyAsync(d_gj, gj.data(), gj.size() * sizeof(double), hipMemcpyHostToDevice, st));
  BZQ_HIP_TRY(hipMemcpyAsync(p->tw_grid, twg.data(), twg.size() * sizeof(double), hipMemcpyHostToDevice, st));
  if (p->fp32)
    BZQ_HIP_TRY(hipMemcpyAsync(p->tw_pad, twpf.data(), twpf.size() * sizeof(float), hipMemcpyHostToDevice, st));
  else
    BZQ_HIP_TRY(hipMemcpyAsync(p->tw_pad, twp.data(), twp.size() * sizeof(double), hipMemcpyHostToDevice, st));
  if (!p->otf) BZQ_HIP_TRY(launch_table(p->V, d_pd, d_gj, p->nj, N, p->npairs, p->fp32, st));
  BZQ_HIP_TRY(hipStreamSynchronize(st));
  return BZQ_OK;
}

enum Stage { ST_PREP = 0, ST_ZINV = 1, ST_PLANE = 2, ST_ZFWD = 3, ST_FINAL = 4, ST_COUNT = 5 };

// Record an event before (begin=true) or after a launch of a timed stage
// (never for a workspace marked untimed, whose calls create nothing).
hipError_t mark(Plan& p, const Workspace& w, int stage, bool begin, hipStream_t st) {
  if (w.untimed || !(p.timing >> stage & 1)) return hipSuccess;
  if (p.ev_used == p.ev_pool.size()) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    p.ev_pool.push_back(e);
  }
  if (begin) p.ev_stage.push_back(stage);
  return hipEventRecord(p.ev_pool[p.ev_used++], st);
}

#define TIMED(stage, expr)                                \
  do {                                                    \
    BZQ_HIP_TRY(mark(p, w, (stage), true, st));           \
    BZQ_HIP_TRY(expr);                                    \
    BZQ_HIP_TRY(mark(p, w, (stage), false, st));          \
  } while (0)

}  // namespace

// Enqueue one evaluation of eq. realQ for `cells` cells of plan p.
bzq_status enqueue_collision(Plan& p, Workspace& w, const PtrPack& f, const PtrPack& Q, int cells,
                             hipStream_t st, const FinUpdate& upd, bool check) {
  if (cells < 1 || cells > w.cells) return fail(BZQ_EINVAL, "more cells than the workspace holds");
  const Geometry g{p.N, p.P};
  CellStrides cs = w.cs;
  cs.cells = cells;
  // a0: the compact spectrum fc (with the NaN/Inf flag when checked), then
  // f(v) on the padded grid, shared by every pair (the copy and the first
  // transform in one launch where they fit)
  int* flag = check ? w.flag : nullptr;
  if (check) BZQ_HIP_TRY(launch_fill_int(w.flag, 0, 1, st));
  if (zinv_ingest_fits(p.P, p.fp32)) {
    TIMED(ST_PREP, launch_zinv_ingest(f, w.fc, w.A, g, p.fp32, cs, st, flag));
  } else {
    TIMED(ST_PREP, launch_ingest(f, w.fc, cs.fc, cells, p.N, p.fp32, st, flag));
  }
  if (check) {
    // nothing that writes an output has been enqueued yet
    int h = 0;
    BZQ_HIP_TRY(hipMemcpyAsync(&h, w.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    BZQ_HIP_TRY(hipStreamSynchronize(st));
    if (h) return fail(BZQ_ENONFINITE, "f_hat holds NaN or Inf (outputs left untouched)");
  }
  if (!zinv_ingest_fits(p.P, p.fp32))
    TIMED(ST_PREP, launch_zinv(w.fc, nullptr, w.A, p.tw_pad, g, 0, 1, ZINV_PLAIN, p.fp32, cs, st));
  TIMED(ST_PREP, launch_plane(w.A, nullptr, nullptr, w.fgrid, p.tw_pad, g, 1, PLANE_TO_GRID, p.fp32, cs, st, 0, w.C));
  // the first last-stage launch writes the S partial accumulators of every
  // cell, later ones add to them
  // the chunk geometry: the plan's, or the workspace's own for scratch of
  // another size
  const int G = w.G ? w.G : p.G, S = w.S ? w.S : p.S, Gw = w.Gw ? w.Gw : p.Gw;
  for (int c0 = 0; c0 < p.npt; c0 += G) {
    const int n = std::min(G, p.npt - c0);
    TIMED(ST_ZINV, launch_zinv(w.fc, p.ph, w.A, p.tw_pad, g, 2 * c0, n, ZINV_PAIRS, p.fp32, cs, st, p.var[0]));
    TIMED(ST_PLANE, launch_plane(w.A, w.B, w.fgrid, nullptr, p.tw_pad, g, n, PLANE_PRODUCT, p.fp32, cs, st,
                                 p.var[1], w.C));
    if (p.otf) {
      // weights of Gw pair-twos at a time, then the last stage over those pair-twos
      for (int w0 = 0; w0 < n; w0 += Gw) {
        const int m = std::min(Gw, n - w0);
        const int pair0 = 2 * (c0 + w0);
        const void* Bw = (const char*)w.B + (size_t)w0 * p.P * 2 * p.nhp * 2 * p.esz;
        TIMED(ST_ZFWD, launch_wgen(w.Vc, p.coef, p.pdv, p.terms, p.mt, p.N, p.Mh, p.nreal, pair0, 2 * m,
                                   p.ncoef, p.fp32, st));
        TIMED(ST_ZFWD, launch_zfwd(Bw, w.Vc, p.ph, p.cp, w.Qpart, p.tw_pad, g, pair0, m, S, p.fp32, cs, st,
                                   p.var[2], pair0, c0 == 0 && w0 == 0));
      }
    } else {
      TIMED(ST_ZFWD, launch_zfwd(w.B, p.V, p.ph, p.cp, w.Qpart, p.tw_pad, g, 2 * c0, n, S, p.fp32, cs, st,
                                 p.var[2], 0, c0 == 0));
    }
  }
  TIMED(ST_FINAL, launch_finalize(w.Qpart, Q, cs.qp, cells, p.N, S, st, upd));
  return BZQ_OK;
}

bzq_status enqueue_step(Plan& p, Workspace& w, const PtrPack& f, int cells, double dt, int n_steps,
                        hipStream_t st, bool check) {
  const size_t n3 = (size_t)p.N * p.N * p.N;
  PtrPack q1{}, q2{}, fs{};
  for (int c = 0; c < cells; ++c) {
    q1.p[c] = w.q1 + c * n3 * 2;
    q2.p[c] = w.q2 + c * n3 * 2;
    fs.p[c] = w.fs + c * n3 * 2;
  }
  // the two updates of the step ride on the finalize launches: fs = f + dt q1
  // with the first evaluation, f += dt/2 (q1 + q2) with the second
  FinUpdate stage, heun;
  stage.mode = FIN_STAGE;
  stage.a = dt;
  stage.ws = w.fs;
  stage.wstride = n3 * 2;
  stage.f = f;
  heun.mode = FIN_HEUN;
  heun.a = 0.5 * dt;
  heun.ws = w.q1;
  heun.wstride = n3 * 2;
  heun.f = f;
  for (int i = 0; i < n_steps; ++i) {
    bzq_status s;
    if ((s = enqueue_collision(p, w, f, q1, cells, st, stage, check && i == 0)) != BZQ_OK) return s;
    if ((s = enqueue_collision(p, w, fs, q2, cells, st, heun)) != BZQ_OK) return s;
  }
  return BZQ_OK;
}

// Classical fourth-order Runge-Kutta: k1 = Q(f), k2 = Q(f + dt/2 k1),
// k3 = Q(f + dt/2 k2), k4 = Q(f + dt k3), f <- f + dt/6 (k1 + 2 k2 + 2 k3 + k4);
// q1 holds the current stage's Q, q2 the running sum, fs the stage argument.
bzq_status enqueue_step_rk4(Plan& p, Workspace& w, const PtrPack& f, int cells, double dt, int n_steps,
                            hipStream_t st, bool check) {
  const size_t n3 = (size_t)p.N * p.N * p.N;
  PtrPack q{}, acc{}, fs{};
  for (int c = 0; c < cells; ++c) {
    q.p[c] = w.q1 + c * n3 * 2;
    acc.p[c] = w.q2 + c * n3 * 2;
    fs.p[c] = w.fs + c * n3 * 2;
  }
  for (int i = 0; i < n_steps; ++i) {
    bzq_status s;
    if ((s = enqueue_collision(p, w, f, q, cells, st, FinUpdate{}, check && i == 0)) != BZQ_OK) return s;
    BZQ_HIP_TRY(launch_axpy_cells(acc, f, dt / 6.0, q, n3, cells, st));
    BZQ_HIP_TRY(launch_axpy_cells(fs, f, 0.5 * dt, q, n3, cells, st));
    if ((s = enqueue_collision(p, w, fs, q, cells, st)) != BZQ_OK) return s;
    BZQ_HIP_TRY(launch_axpy_cells(acc, acc, dt / 3.0, q, n3, cells, st));
    BZQ_HIP_TRY(launch_axpy_cells(fs, f, 0.5 * dt, q, n3, cells, st));
    if ((s = enqueue_collision(p, w, fs, q, cells, st)) != BZQ_OK) return s;
    BZQ_HIP_TRY(launch_axpy_cells(acc, acc, dt / 3.0, q, n3, cells, st));
    BZQ_HIP_TRY(launch_axpy_cells(fs, f, dt, q, n3, cells, st));
    if ((s = enqueue_collision(p, w, fs, q, cells, st)) != BZQ_OK) return s;
    BZQ_HIP_TRY(launch_axpy_cells(f, acc, dt / 6.0, q, n3, cells, st));
  }
  return BZQ_OK;
}

bzq_status create_plan(bzq_plan* out, int N, double L, double R, double gamma, double bc, double bs,
                       double br, int nj, int N_rho, int M, int precision, void* stream, bool otf, int kind,
                       double theta_cut) {
  if (!out) return fail(BZQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (N < 8 || (N & 1)) return fail(BZQ_EINVAL, "N must be even and >= 8");
  if (!(L > 0) || !std::isfinite(L)) return fail(BZQ_EINVAL, "L must be > 0");
  if (!(R > 0) || !std::isfinite(R)) return fail(BZQ_EINVAL, "R must be > 0");
  if (!(gamma > -3.0 && gamma <= 1.0)) return fail(BZQ_EINVAL, "gamma must lie in (-3, 1]");
  if (!(bs >= -1.0 && bs < 1.0)) return fail(BZQ_EINVAL, "s must lie in [-1, 1) (in [0, 1) for the power kernel)");
  if (!(br >= 0.0 && br < 1.0)) return fail(BZQ_EINVAL, "r must lie in [0, 1)");
  if (!(bc > 0) || !std::isfinite(bc)) return fail(BZQ_EINVAL, "kernel constant c must be > 0");
  if (nj < 8 || nj > 256) return fail(BZQ_EINVAL, "n_jacobi must lie in [8, 256]");
  if (N_rho < 1 || N_rho > 4096) return fail(BZQ_EINVAL, "N_rho must lie in [1, 4096]");
  if (precision != BZQ_FP64 && precision != BZQ_FP32_ACC64) return fail(BZQ_EINVAL, "unknown precision");
  std::vector<double> tmp;
  if (!lebedev_rule(M, tmp)) return fail(BZQ_EINVAL, "M is not the size of an available Lebedev rule");
  if (!supported_N(N)) return fail(BZQ_EUNSUPPORTED, "no FFT schedule for this N (supported: 8 16 24 32 48 64 128)");
  bzq_plan_s* p = new bzq_plan_s();
  p->N = N;
  p->P = 3 * N / 2;
  p->n1 = N - 1;
  p->nn = p->n1 * p->n1;
  p->nh = (p->nn + 1) / 2;
  p->L = L; p->R = R; p->gamma = gamma;
  p->bc = bc; p->bs = bs; p->br = br; p->nj = nj;
  p->N_rho = N_rho; p->M = M;
  p->fp32 = precision == BZQ_FP32_ACC64;
  p->otf = otf;
  p->kind = kind;
  p->theta_cut = theta_cut;
  bzq_status s = build_plan(p, (hipStream_t)stream);
  if (s != BZQ_OK) {
    delete p;
    return s;
  }
  *out = p;
  return BZQ_OK;
}

double power_kernel_constant(double s) { return (1.0 - s) * (2.0 - s) / (24.0 * (double)kPi); }

// (c, s, r) of b = c t^{-1-s} (1-t)^{-r} for a bzq_kernel selector: the power
// kernel c_s t^{-1-s} (0 <= s < 1), the constant cutoff kernel 1/(4 pi)
// (= c t^{-1-s} with s = -1: b5 of Section 5.3), or (when `general` is
// allowed) the explicit triple.
bzq_status kernel_params(int kernel, double s, double c, double r, bool general, double* bc, double* bs,
                         double* br) {
  switch (kernel) {
    case BZQ_KERNEL_POWER:
      if (!(s >= 0.0 && s < 1.0)) return fail(BZQ_EINVAL, "s must lie in [0, 1)");
      *bc = power_kernel_constant(s);
      *bs = s;
      *br = 0.0;
      return BZQ_OK;
    case BZQ_KERNEL_CUTOFF_CONST:
      *bc = (double)(1.0L / (4.0L * kPi));
      *bs = -1.0;
      *br = 0.0;
      return BZQ_OK;
    case BZQ_KERNEL_GENERAL:
      if (!general) break;
      *bc = c;
      *bs = s;
      *br = r;
      return BZQ_OK;
    default:
      break;
  }
  return fail(BZQ_EINVAL, "unknown angular kernel selector");
}

namespace {

// f on the physical N^3 grid (FP64) into dst, layout [z][x][y]
bzq_status enqueue_to_grid(Plan& p, const double* f_hat, double* dst, hipStream_t st) {
  const Geometry g{p.N, p.N};
  CellStrides cs{};
  cs.cells = 1;
  BZQ_HIP_TRY(launch_ingest(single(f_hat), p.gfc, 0, 1, p.N, false, st));
  BZQ_HIP_TRY(launch_zinv(p.gfc, nullptr, p.gA, p.tw_grid, g, 0, 1, ZINV_GRID_SIGN, false, cs, st));
  cs.pc = (size_t)p.N * p.n1 * p.N;
  BZQ_HIP_TRY(launch_plane(p.gA, nullptr, nullptr, dst, p.tw_grid, g, 1, PLANE_TO_GRID, false, cs, st, 0, p.gC));
  return BZQ_OK;
}

}  // namespace
}  // namespace bzq

using namespace bzq;

struct bzq_workspace_s : bzq::Workspace {};

extern "C" {

bzq_status bzq_plan_create(bzq_plan* out, int N, double L, double R, double gamma, double s, int N_rho, int M,
                           int precision, int kernel, void* stream) {
  double bc = 0, bs = 0, br = 0;
  const bzq_status ks = kernel_params(kernel, s, 0.0, 0.0, false, &bc, &bs, &br);
  if (ks != BZQ_OK) {
    if (out) *out = nullptr;
    return ks;
  }
  return create_plan(out, N, L, R, gamma, bc, bs, br, 64, N_rho, M, precision, stream);
}

bzq_status bzq_plan_create_general(bzq_plan* out, int N, double L, double R, double gamma, double b_c,
                                   double b_s, double b_r, int n_jacobi, int N_rho, int M, int precision,
                                   void* stream) {
  return create_plan(out, N, L, R, gamma, b_c, b_s, b_r, n_jacobi, N_rho, M, precision, stream);
}

bzq_status bzq_plan_create_debye(bzq_plan* out, int N, double L, double R, double theta_cut, int N_rho, int M,
                                 int precision, void* stream) {
  if (!(theta_cut >= 0.0 && theta_cut < (double)(kPi / 3))) {
    if (out) *out = nullptr;
    return fail(BZQ_EINVAL, "theta_cut must lie in [0, pi/3)");
  }
  return create_plan(out, N, L, R, 1.0, 0.25, 0.0, 0.0, 64, N_rho, M, precision, stream, false, 1, theta_cut);
}

bzq_status bzq_plan_create_otf(bzq_plan* out, int N, double L, double R, double gamma, int kernel, double b_c,
                               double b_s, double b_r, int N_rho, int M, int precision, void* stream) {
  double bc = 0, bs = 0, br = 0;
  const bzq_status ks = kernel_params(kernel, b_s, b_c, b_r, true, &bc, &bs, &br);
  if (ks != BZQ_OK) {
    if (out) *out = nullptr;
    return ks;
  }
  return create_plan(out, N, L, R, gamma, bc, bs, br, 64, N_rho, M, precision, stream, true);
}

bzq_status bzq_plan_derive_gamma(bzq_plan* out, bzq_plan base, double gamma, void* stream) {
  if (!base) {
    if (out) *out = nullptr;
    return fail(BZQ_EINVAL, "NULL base plan");
  }
  return derive_plan(*base, gamma, out, (hipStream_t)stream);
}

size_t bzq_plan_shared_bytes(bzq_plan p) { return p ? p->shared->bytes : 0; }

bzq_status bzq_collision(bzq_plan p, const double* f_hat, double* Q_hat, void* stream) {
  if (!p || !f_hat || !Q_hat) return fail(BZQ_EINVAL, "NULL argument");
  if (ranges_overlap(f_hat, Q_hat, state_bytes(p->N))) return fail(BZQ_EINVAL, "f_hat and Q_hat must not overlap");
  return enqueue_collision(*p, p->ws, single(f_hat), single(Q_hat), 1, (hipStream_t)stream, FinUpdate{}, true);
}

bzq_status bzq_collision_noalloc(bzq_plan p, const double* f_hat, double* Q_hat, void* stream) {
  if (!p || !f_hat || !Q_hat) return fail(BZQ_EINVAL, "NULL argument");
  if (ranges_overlap(f_hat, Q_hat, state_bytes(p->N))) return fail(BZQ_EINVAL, "f_hat and Q_hat must not overlap");
  // the largest chunk of pair-twos (at most the plan's) whose scratch fits
  const size_t esz = p->esz;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t b_fc = al((size_t)p->n1 * p->nn * 2 * esz), b_fg = al((size_t)p->P * p->P * p->P * esz);
  const int zv = effective_variant(*p, 2);
  int G = p->G, S = 0, Gw = 0;
  size_t b_a = 0, b_b = 0, b_c = 0, b_q = 0, b_w = 0;
  auto need = [&](int g) {
    S = zfwd_splits_for(*p, g, zv, p->s_target);
    Gw = p->otf ? std::min(p->Gw, g) : 0;
    b_a = al((size_t)g * p->P * a_plane(p->N) * 2 * esz);
    b_b = al((size_t)g * p->P * 2 * p->nhp * 2 * esz);
    b_c = al(plane_rows_elems(*p, g) * 2 * esz);
    b_q = al((size_t)S * p->nh * p->n1 * 16);
    b_w = al((size_t)2 * Gw * weight_row(p->N) * p->n1 * esz);
    return b_fc + b_fg + b_a + b_b + b_c + b_q + b_w;
  };
  while (G > 1 && need(G) > kNoAllocScratchBytes) --G;
  if (need(G) > kNoAllocScratchBytes)
    return fail(BZQ_EUNSUPPORTED, "plan too large for the no-allocation scratch (" +
                                      std::to_string(need(G)) + " bytes needed, " +
                                      std::to_string(kNoAllocScratchBytes) + " available)");
  void* base = nullptr;
  BZQ_HIP_TRY(noalloc_scratch(&base));
  // a workspace that owns nothing: its buffers are slices of the scratch
  Workspace w;
  w.plan = p;
  w.cells = 1;
  w.G = G;
  w.S = S;
  w.Gw = Gw;
  w.untimed = true;
  char* at = (char*)base;
  w.fc = at; at += b_fc;
  w.fgrid = at; at += b_fg;
  w.A = at; at += b_a;
  w.B = at; at += b_b;
  w.C = b_c ? at : nullptr; at += b_c;
  w.Qpart = (double*)at; at += b_q;
  w.Vc = p->otf ? at : nullptr;
  w.cs.fc = (size_t)p->n1 * p->nn;
  w.cs.fg = (size_t)p->P * p->P * p->P;
  w.cs.a = (size_t)G * p->P * a_plane(p->N);
  w.cs.b = (size_t)G * p->P * 2 * p->nhp;
  w.cs.qp = (size_t)S * p->nh * p->n1;
  w.cs.pc = plane_rows_elems(*p, G);
  w.cs.cells = 1;
  return enqueue_collision(*p, w, single(f_hat), single(Q_hat), 1, (hipStream_t)stream);
}

bzq_status bzq_step(bzq_plan p, double* f_hat, double dt, int n_steps, void* stream) {
  if (!p || !f_hat) return fail(BZQ_EINVAL, "NULL argument");
  if (!std::isfinite(dt) || n_steps < 0) return fail(BZQ_EINVAL, "bad dt or n_steps");
  if (n_steps == 0) return BZQ_OK;
  return enqueue_step(*p, p->ws, single(f_hat), 1, dt, n_steps, (hipStream_t)stream, true);
}

namespace {

int encode_schedule(const Plan& p) {
  int t = 0;
  while (t < 2 && kSTargets[t] != p.s_target) ++t;
  return p.var[0] | p.var[1] << 2 | p.var[2] << 4 | t << 6;
}
void decode_schedule(Plan& p, int code) {
  p.var[0] = code & 3;
  p.var[1] = code >> 2 & 3;
  p.var[2] = code >> 4 & 3;
  p.s_target = kSTargets[std::min(2, code >> 6 & 3)];
}
std::string schedule_key(const Plan& p) {
  std::ostringstream k;
  k << "schedule N=" << p.N << " P=" << p.P << " prec=" << (p.fp32 ? "fp32" : "fp64")
    << " npairs=" << p.npairs << " G=" << p.G << (p.otf ? " otf" : "");
  return k.str();
}

// Best of four timed evaluations (after one untimed) with the plan's current
// schedule, in milliseconds.
bzq_status time_schedule(Plan& p, const double* f_hat, double* Q, hipStream_t st, float* best) {
  hipEvent_t e0, e1;
  BZQ_HIP_TRY(hipEventCreate(&e0));
  BZQ_HIP_TRY(hipEventCreate(&e1));
  bzq_status s = enqueue_collision(p, p.ws, single(f_hat), single(Q), 1, st);
  *best = 1e30f;
  for (int r = 0; r < 4 && s == BZQ_OK; ++r) {
    (void)hipEventRecord(e0, st);
    s = enqueue_collision(p, p.ws, single(f_hat), single(Q), 1, st);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) s = fail(BZQ_EDEVICE, "timing an evaluation failed");
    float ms = 0.f;
    if (s == BZQ_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) *best = std::min(*best, ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return s;
}

}  // namespace

bzq_status bzq_plan_set_schedule(bzq_plan p, const int* sched) {
  if (!p || !sched) return fail(BZQ_EINVAL, "NULL argument");
  for (int st = 0; st < 3; ++st) {
    const int v = sched[st];
    if (v < 0 || v > 3 || (v && !(stage_variants(st, p->P, p->fp32) >> v & 1)))
      return fail(BZQ_EINVAL, "kernel variant not available for this plan");
  }
  if (sched[3] != kSTargets[0] && sched[3] != kSTargets[1] && sched[3] != kSTargets[2])
    return fail(BZQ_EINVAL, "s_target must be 512, 1024 or 2048");
  const int G = p->G, S_cap = p->S_cap;
  for (int st = 0; st < 3; ++st) p->var[st] = sched[st];
  p->s_target = sched[3];
  set_chunking(*p);
  if (p->G != G || p->S_cap != S_cap) return fail(BZQ_EDEVICE, "schedule changed the workspace geometry");
  return BZQ_OK;
}

bzq_status bzq_plan_schedule(bzq_plan p, int* out) {
  if (!p || !out) return fail(BZQ_EINVAL, "NULL argument");
  for (int st = 0; st < 3; ++st) out[st] = effective_variant(*p, st);
  out[3] = p->s_target;
  out[4] = p->S;
  return BZQ_OK;
}

bzq_status bzq_plan_autotune(bzq_plan p, const double* f_hat, int use_cache, void* stream) {
  if (!p || !f_hat) return fail(BZQ_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  const std::string key = schedule_key(*p);
  if (use_cache) {
    auto cache = tune_cache_read();
    auto it = cache.find(key);
    if (it != cache.end()) {
      decode_schedule(*p, it->second);
      set_chunking(*p);
      return BZQ_OK;
    }
  }
  double* Q = p->ws.q1;   // scratch output (the workspace is idle between calls)
  float best = 0.f;
  bzq_status s = time_schedule(*p, f_hat, Q, st, &best);
  if (s != BZQ_OK) return s;
  // one stage at a time, the others kept at their best so far
  for (int stage = 0; stage < 3; ++stage) {
    const unsigned avail = stage_variants(stage, p->P, p->fp32);
    for (int v = 1; v <= 3; ++v) {
      for (int t = 0; t < 3; ++t) {
        if (!(avail >> v & 1)) continue;
        if (stage < 2 && t != 1) continue;   // s_target matters to the z-forward only
        const int old_v = p->var[stage], old_t = p->s_target;
        if (effective_variant(*p, stage) == v && (stage < 2 || kSTargets[t] == old_t)) continue;
        p->var[stage] = v;
        if (stage == 2) p->s_target = kSTargets[t];
        set_chunking(*p);
        float ms = 0.f;
        if ((s = time_schedule(*p, f_hat, Q, st, &ms)) != BZQ_OK) return s;
        if (ms < 0.97f * best) {   // a candidate must win clearly over timing noise
          best = ms;
        } else {
          p->var[stage] = old_v;
          p->s_target = old_t;
          set_chunking(*p);
        }
      }
    }
  }
  for (int stage = 0; stage < 3; ++stage) p->var[stage] = effective_variant(*p, stage);
  set_chunking(*p);
  auto cache = tune_cache_read();
  cache[key] = encode_schedule(*p);
  tune_cache_write(cache);
  return BZQ_OK;
}

bzq_status bzq_step_rk4(bzq_plan p, double* f_hat, double dt, int n_steps, void* stream) {
  if (!p || !f_hat) return fail(BZQ_EINVAL, "NULL argument");
  if (!std::isfinite(dt) || n_steps < 0) return fail(BZQ_EINVAL, "bad dt or n_steps");
  if (n_steps == 0) return BZQ_OK;
  return enqueue_step_rk4(*p, p->ws, single(f_hat), 1, dt, n_steps, (hipStream_t)stream, true);
}

bzq_status bzq_workspace_create(bzq_workspace* out, bzq_plan p) {
  if (!out || !p) return fail(BZQ_EINVAL, "NULL argument");
  *out = nullptr;
  auto* w = new bzq_workspace_s();
  bzq_status s = workspace_init(*w, *p, 1);
  if (s != BZQ_OK) {
    delete w;
    return s;
  }
  *out = w;
  return BZQ_OK;
}

bzq_status bzq_collision_ws(bzq_plan p, bzq_workspace w, const double* f_hat, double* Q_hat, void* stream) {
  if (!p || !w || !f_hat || !Q_hat) return fail(BZQ_EINVAL, "NULL argument");
  if (w->plan != p) return fail(BZQ_EINVAL, "workspace was made for another plan");
  if (ranges_overlap(f_hat, Q_hat, state_bytes(p->N))) return fail(BZQ_EINVAL, "f_hat and Q_hat must not overlap");
  return enqueue_collision(*p, *w, single(f_hat), single(Q_hat), 1, (hipStream_t)stream, FinUpdate{}, true);
}

bzq_status bzq_step_ws(bzq_plan p, bzq_workspace w, double* f_hat, double dt, int n_steps, void* stream) {
  if (!p || !w || !f_hat) return fail(BZQ_EINVAL, "NULL argument");
  if (w->plan != p) return fail(BZQ_EINVAL, "workspace was made for another plan");
  if (!std::isfinite(dt) || n_steps < 0) return fail(BZQ_EINVAL, "bad dt or n_steps");
  if (n_steps == 0) return BZQ_OK;
  return enqueue_step(*p, *w, single(f_hat), 1, dt, n_steps, (hipStream_t)stream, true);
}

size_t bzq_workspace_bytes(bzq_workspace w) { return w ? w->arena.bytes : 0; }

bzq_status bzq_workspace_destroy(bzq_workspace w) {
  if (!w) return BZQ_OK;
  (void)hipDeviceSynchronize();
  delete w;
  return BZQ_OK;
}

bzq_status bzq_moments(bzq_plan p, const double* f_hat, const double* Q_hat, double* out, void* stream) {
  if (!p || !f_hat || !out) return fail(BZQ_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  bzq_status s;
  const double* q = Q_hat;
  if (!q) {
    if ((s = enqueue_collision(*p, p->ws, single(f_hat), single(p->ws.q1), 1, st)) != BZQ_OK) return s;
    q = p->ws.q1;
  }
  if ((s = enqueue_to_grid(*p, f_hat, p->gf, st)) != BZQ_OK) return s;
  if ((s = enqueue_to_grid(*p, q, p->gq, st)) != BZQ_OK) return s;
  BZQ_HIP_TRY(launch_moments(p->gf, nullptr, -1.0, p->L, p->N, p->part, kMomentBlocks, st));
  std::vector<double> part((size_t)kMomentBlocks * 8);
  double f0[2];
  BZQ_HIP_TRY(hipMemcpyAsync(part.data(), p->part, part.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  BZQ_HIP_TRY(hipMemcpyAsync(f0, f_hat, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  BZQ_HIP_TRY(hipStreamSynchronize(st));
  double sums[5] = {0, 0, 0, 0, 0}, fmax = -1e300;
  for (int b = 0; b < kMomentBlocks; ++b) {
    for (int k = 0; k < 5; ++k) sums[k] += part[b * 8 + k];
    fmax = std::max(fmax, part[b * 8 + 5]);
  }
  BZQ_HIP_TRY(launch_moments(p->gf, p->gq, 1e-14 * std::max(fmax, 0.0), p->L, p->N, p->part, kMomentBlocks, st));
  BZQ_HIP_TRY(hipMemcpyAsync(part.data(), p->part, part.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  BZQ_HIP_TRY(hipStreamSynchronize(st));
  double ent = 0;
  for (int b = 0; b < kMomentBlocks; ++b) ent += part[b * 8 + 6];
  const double h3 = std::pow(2.0 * p->L / p->N, 3);
  out[0] = std::pow(2.0 * p->L, 3) * f0[0];
  out[1] = h3 * sums[1];
  out[2] = h3 * sums[2];
  out[3] = h3 * sums[3];
  out[4] = h3 * sums[4];
  out[5] = h3 * ent;
  return BZQ_OK;
}

bzq_status bzq_check_finite(bzq_plan p, const double* f_hat, void* stream) {
  if (!p || !f_hat) return fail(BZQ_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  int h = 0;
  BZQ_HIP_TRY(hipMemcpyAsync(p->flag, &h, sizeof(int), hipMemcpyHostToDevice, st));
  BZQ_HIP_TRY(launch_finite(f_hat, (size_t)p->N * p->N * p->N * 2, p->flag, st));
  BZQ_HIP_TRY(hipMemcpyAsync(&h, p->flag, sizeof(int), hipMemcpyDeviceToHost, st));
  BZQ_HIP_TRY(hipStreamSynchronize(st));
  return h ? fail(BZQ_ENONFINITE, "f_hat holds NaN or Inf") : BZQ_OK;
}

size_t bzq_plan_device_bytes(bzq_plan p) {
  return p ? p->shared->bytes + p->tables.bytes + p->ws.arena.bytes + p->grid_scratch.bytes : 0;
}

size_t bzq_plan_bytes_estimate(int N, int N_rho, int M, int precision) {
  if (N < 8 || (N & 1) || N_rho < 1 || M < 6) return 0;
  return plan_footprint(N, N_rho, M, precision);
}

size_t bzq_request_device_bytes(int N, int precision) {
  if (N < 8 || (N & 1) || (precision != BZQ_FP64 && precision != BZQ_FP32_ACC64)) return 0;
  // a workspace of any plan of this N: the chunk of pair-twos saturates at its
  // cap for many pairs, so a plan with very many pairs bounds every other
  Plan p;
  p.N = N;
  p.P = 3 * N / 2;
  p.n1 = N - 1;
  p.nn = p.n1 * p.n1;
  p.nh = (p.nn + 1) / 2;
  p.fp32 = precision == BZQ_FP32_ACC64;
  p.npairs = 1 << 24;
  p.npt = p.npairs / 2;
  set_chunking(p);
  return 2 * state_bytes(N) + p.workspace_bytes_per_cell();
}

bzq_status bzq_plan_info(bzq_plan p, double* out) {
  if (!p || !out) return fail(BZQ_EINVAL, "NULL argument");
  out[0] = p->N;
  out[1] = p->P;
  out[2] = p->npairs;
  out[3] = 2.0 * p->G;
  out[4] = p->S;
  out[5] = p->fp32 ? BZQ_FP32_ACC64 : BZQ_FP64;
  out[6] = p->nj;
  out[7] = p->otf ? (double)((size_t)p->N_rho * p->mt * p->ncoef * sizeof(double))
                  : (double)((size_t)p->npairs * weight_row(p->N) * p->n1 * p->esz);
  return BZQ_OK;
}

bzq_status bzq_plan_pairs(bzq_plan p, double* out) {
  if (!p || !out) return fail(BZQ_EINVAL, "NULL argument");
  std::memcpy(out, p->pair_host.data(), p->pair_host.size() * sizeof(double));
  return BZQ_OK;
}

bzq_status bzq_plan_weights(bzq_plan p, int pair, double* out) {
  if (!p || !out) return fail(BZQ_EINVAL, "NULL argument");
  if (pair < 0 || pair >= p->npairs) return fail(BZQ_EINVAL, "pair index out of range");
  // stored as [i3][c] (rows of weight_row(N) entries); returned as [c][i3]
  const int nhv = weight_row(p->N);
  const size_t cnt = (size_t)nhv * p->n1;
  const char* src = nullptr;
  DeviceArena scratch;
  if (!p->otf) {
    src = (const char*)p->V + (size_t)pair * cnt * p->esz;
  } else {
    // evaluate this pair's weights with the kernel the evaluations use
    void* d = nullptr;
    bzq_status s = scratch.get(&d, cnt * p->esz);
    if (s != BZQ_OK) return s;
    BZQ_HIP_TRY(launch_wgen(d, p->coef, p->pdv, p->terms, p->mt, p->N, p->Mh, p->nreal, pair, 1, p->ncoef,
                            p->fp32, nullptr));
    BZQ_HIP_TRY(hipStreamSynchronize(nullptr));
    src = (const char*)d;
  }
  std::vector<double> tmp(cnt);
  if (p->fp32) {
    std::vector<float> tf(cnt);
    BZQ_HIP_TRY(hipMemcpy(tf.data(), src, cnt * sizeof(float), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < cnt; ++i) tmp[i] = tf[i];
  } else {
    BZQ_HIP_TRY(hipMemcpy(tmp.data(), src, cnt * sizeof(double), hipMemcpyDeviceToHost));
  }
  for (int i3 = 0; i3 < p->n1; ++i3)
    for (int c = 0; c < p->nh; ++c) out[(size_t)c * p->n1 + i3] = tmp[(size_t)i3 * nhv + c];
  return BZQ_OK;
}

bzq_status bzq_plan_set_timing(bzq_plan p, int enable) {
  if (!p) return fail(BZQ_EINVAL, "NULL plan");
  if (enable < 0) return fail(BZQ_EINVAL, "timing mask must be >= 0");
  p->timing = enable == 1 ? (1 << ST_COUNT) - 1 : enable;
  p->ev_stage.clear();
  p->ev_used = 0;
  return BZQ_OK;
}

bzq_status bzq_plan_stage_times(bzq_plan p, double* out) {
  if (!p || !out) return fail(BZQ_EINVAL, "NULL argument");
  for (int i = 0; i < 2 * ST_COUNT; ++i) out[i] = 0.0;
  for (size_t i = 0; i < p->ev_stage.size(); ++i) {
    BZQ_HIP_TRY(hipEventSynchronize(p->ev_pool[2 * i + 1]));
    float ms = 0.f;
    BZQ_HIP_TRY(hipEventElapsedTime(&ms, p->ev_pool[2 * i], p->ev_pool[2 * i + 1]));
    out[p->ev_stage[i]] += ms;
    out[ST_COUNT + p->ev_stage[i]] += 1.0;
  }
  p->ev_stage.clear();
  p->ev_used = 0;
  return BZQ_OK;
}

bzq_status bzq_plan_destroy(bzq_plan p) {
  if (!p) return BZQ_OK;
  (void)hipDeviceSynchronize();
  delete p;
  return BZQ_OK;
}

const char* bzq_status_string(bzq_status s) {
  switch (s) {
    case BZQ_OK: return "ok";
    case BZQ_EINVAL: return "invalid argument";
    case BZQ_ENOMEM: return "out of device memory";
    case BZQ_EDEVICE: return "HIP runtime error";
    case BZQ_EUNSUPPORTED: return "unsupported size";
    case BZQ_ENONFINITE: return "non-finite input";
    case BZQ_EBUSY: return "request queue full";
  }
  return "unknown status";
}

const char* bzq_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
