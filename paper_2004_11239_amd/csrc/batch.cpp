// Batched executor: many independent homogeneous cells, each with its own
// f_hat, advanced together.  Cells that share a plan (same N, L, R, gamma,
// kernel, quadrature and precision) share its weight tables and run in the
// same launches, stacked along the grid's third dimension (up to 64 cells per
// launch); the kernels, chunking and accumulation order per cell are those of
// a single evaluation, so every cell's result is bitwise identical to
// bzq_collision / bzq_step on its own.
//
// Cells per launch are chosen per plan by a small autotuner (time one
// evaluation of each candidate count on the batch's own data, keep the
// fastest per-cell time) whose choices persist in a text cache keyed by the
// plan geometry.  A whole Heun step of the batch can be captured once into a
// HIP graph and replayed.
//
// Mixed sizes in one launch (switched off, see kMixedLaunches): when every
// plan of the batch is an FP32 table plan with N in {16, 24, 32} and the
// kernel variants of the mixed launches, the cells of all sizes run together,
// round after round: a round holds, for each size, as many cells as it has
// workspace slots (slots sized so that all sizes finish in the same number of
// rounds within the workspace budget), and each pipeline stage of a round is
// one launch over a device table of (cell, workgroup) items of every size
// (launch_mix).  Per cell the kernels' bodies, arguments and order are those
// of the single-cell path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <memory>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "plan.hpp"

namespace bzq {
namespace {

struct Group {
  Plan* plan = nullptr;
  std::vector<int> cells;   // indices into the batch's cell list
  int cpl = 1;              // cells per launch
  bool tuned = false;       // cpl came from timing (not from the cache or the caller)
  Workspace* ws = nullptr;
};

std::string tune_key(const Plan& p) {
  std::ostringstream k;
  k << "N=" << p.N << " P=" << p.P << " prec=" << (p.fp32 ? "fp32" : "fp64") << " npairs=" << p.npairs
    << " G=" << p.G << " S=" << p.S << " sched=" << p.var[0] << p.var[1] << p.var[2] << (p.otf ? " otf" : "");
  return k.str();
}

size_t ws_budget_bytes() {
  const char* e = std::getenv("BZQ_BATCH_WS_MB");
  const size_t mb = e ? (size_t)std::atoll(e) : 8192;
  return mb << 20;
}

}  // namespace
}  // namespace bzq

using namespace bzq;

// Rounds of the mixed-size launches: slot workspaces, the per-round cell
// tables and work-item offsets on the device.
struct MixedRounds {
  std::vector<Workspace*> slot_ws;            // one cell each
  std::vector<int> slot_group;                // group of each slot
  int rounds = 0, max_cells = 0;
  std::vector<int> ncells;                    // active cells per round
  std::vector<std::array<int, MIX_STAGES>> totals;   // items per (round, stage)
  MixCell* d_cells = nullptr;                 // [round][max_cells]
  int* d_offs = nullptr;                      // [round][stage][max_cells + 1]
  double2** d_outs = nullptr;                 // [cell] outputs of bzq_batch_collision
  std::vector<double*> h_outs;
  DeviceArena arena;
  ~MixedRounds() {
    for (Workspace* w : slot_ws) delete w;
  }
};

struct bzq_batch_s {
  std::vector<double*> f;
  std::vector<Group> groups;
  std::unique_ptr<MixedRounds> mix;   // set when the cells run in mixed-size launches
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;   // private stream the graph is recorded on
  double graph_dt = 0.0;

  ~bzq_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (capture) (void)hipStreamDestroy(capture);
    for (auto& g : groups) delete g.ws;
  }
};

namespace {

PtrPack pack(const std::vector<double*>& ptrs, const std::vector<int>& idx, size_t from, int n) {
  PtrPack pk{};
  for (int i = 0; i < n; ++i) pk.p[i] = ptrs[idx[from + i]];
  return pk;
}

// time one evaluation of `n` cells of group g with `cpl` cells per launch
// (best of three after a warm-up): at least 64 cells (or all of them), so
// that candidates a few per cent apart are told apart (over two launches'
// worth of cells, once, the choice at 16^3 and 24^3 fell on 8 and 4 cells
// per launch, 3 and 4.5 % slower per batch step than 16)
bzq_status time_candidate(Group& g, const std::vector<double*>& f, int cpl, hipStream_t st, float* ms_per_cell) {
  Workspace w;
  bzq_status s = workspace_init(w, *g.plan, cpl);
  if (s != BZQ_OK) return s;
  const int n = std::min<int>((int)g.cells.size(), std::max(2 * cpl, 64));
  const size_t n3 = (size_t)g.plan->N * g.plan->N * g.plan->N;
  hipEvent_t e0, e1;
  BZQ_HIP_TRY(hipEventCreate(&e0));
  BZQ_HIP_TRY(hipEventCreate(&e1));
  auto run = [&]() -> bzq_status {
    for (int c0 = 0; c0 < n; c0 += cpl) {
      const int m = std::min(cpl, n - c0);
      PtrPack out{};
      for (int i = 0; i < m; ++i) out.p[i] = w.q1 + i * n3 * 2;
      bzq_status r = enqueue_collision(*g.plan, w, pack(f, g.cells, c0, m), out, m, st);
      if (r != BZQ_OK) return r;
    }
    return BZQ_OK;
  };
  const bool timing = g.plan->timing;
  g.plan->timing = false;
  s = run();   // warm-up
  float ms = 0;
  for (int rep = 0; rep < 3 && s == BZQ_OK; ++rep) {
    (void)hipEventRecord(e0, st);
    s = run();
    (void)hipEventRecord(e1, st);
    float t = 0;
    if (s == BZQ_OK) {
      (void)hipEventSynchronize(e1);
      (void)hipEventElapsedTime(&t, e0, e1);
      ms = rep == 0 ? t : std::min(ms, t);
    }
  }
  g.plan->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  *ms_per_cell = ms / n;
  return s;
}

bzq_status autotune(Group& g, const std::vector<double*>& f, hipStream_t st) {
  auto cache = tune_cache_read();
  const std::string key = tune_key(*g.plan);
  auto it = cache.find(key);
  const int ncell = (int)g.cells.size();
  const size_t per_cell = g.plan->workspace_bytes_per_cell();
  const int mem_cap = (int)std::max<size_t>(1, ws_budget_bytes() / per_cell);
  if (it != cache.end() && it->second >= 1) {
    g.cpl = std::max(1, std::min({it->second, ncell, kMaxCells, mem_cap}));
    return BZQ_OK;
  }
  int best = 1;
  float best_ms = 1e30f;
  for (int c : {1, 2, 4, 8, 16, 32, 64}) {
    if (c > ncell || c > mem_cap || c > kMaxCells) break;
    float ms = 0;
    bzq_status s = time_candidate(g, f, c, st, &ms);
    if (s == BZQ_ENOMEM) break;
    if (s != BZQ_OK) return s;
    if (ms < best_ms * 0.99f) {   // more cells per launch only for a clear gain
      best_ms = ms;
      best = c;
    }
  }
  g.cpl = best;
  g.tuned = true;
  if (ncell >= 2 * best) {   // only a choice made with room to spare is worth caching
    cache[key] = best;
    tune_cache_write(cache);
  }
  return BZQ_OK;
}

// Phase `phase` of round r in mixed-size launches (phase 0: Q into the
// batch's outputs; 1, 2: the two evaluations of a Heun step).
bzq_status enqueue_mixed_round(bzq_batch_s* b, int r, int phase, double a, hipStream_t st) {
  MixedRounds& m = *b->mix;
  const MixCell* cells = m.d_cells + (size_t)r * m.max_cells;
  for (int stg = 0; stg < MIX_STAGES; ++stg) {
    const int* offs = m.d_offs + ((size_t)r * MIX_STAGES + stg) * (m.max_cells + 1);
    BZQ_HIP_TRY(launch_mix(stg, cells, offs, m.ncells[r], m.totals[r][stg], phase, a, m.d_outs, st));
  }
  return BZQ_OK;
}

// One evaluation (step = false) or one Heun step of every cell, round after
// round.  Both evaluations of a step finish within the round: the next round
// reuses the slots' stage buffers (fs, q1).
bzq_status enqueue_mixed(bzq_batch_s* b, bool step, double dt, hipStream_t st) {
  for (int r = 0; r < b->mix->rounds; ++r) {
    bzq_status s = enqueue_mixed_round(b, r, step ? 1 : 0, dt, st);
    if (s == BZQ_OK && step) s = enqueue_mixed_round(b, r, 2, 0.5 * dt, st);
    if (s != BZQ_OK) return s;
  }
  return BZQ_OK;
}

bzq_status enqueue_batch_step(bzq_batch_s* b, double dt, hipStream_t st) {
  if (b->mix) return enqueue_mixed(b, true, dt, st);
  for (auto& g : b->groups) {
    for (size_t c0 = 0; c0 < g.cells.size(); c0 += g.cpl) {
      const int m = (int)std::min<size_t>(g.cpl, g.cells.size() - c0);
      bzq_status s = enqueue_step(*g.plan, *g.ws, pack(b->f, g.cells, c0, m), m, dt, 1, st);
      if (s != BZQ_OK) return s;
    }
  }
  return BZQ_OK;
}

// The mixed-size launches are switched off: their first run on the device
// ended in a GPU memory fault whose cause is not known.  Until it is, batches
// run in groups of one plan each and cells_per_launch = -1 is refused.
constexpr bool kMixedLaunches = false;

// Whether every group runs in the mixed-size launches.
bool mixed_eligible(const bzq_batch_s* b) {
  for (const auto& g : b->groups) {
    const Plan& p = *g.plan;
    if (p.otf || p.G != p.npt) return false;
    if (!mix_supported(p.N, p.fp32, effective_variant(p, 0), effective_variant(p, 1), effective_variant(p, 2)))
      return false;
  }
  return true;
}

// Rounds for the mixed-size launches: the fewest rounds R for which a slot
// per ceil(cells / R) cells of every size fits the workspace budget; cells of
// the largest N first in each round's table (their items are the heaviest).
bzq_status plan_mixed(bzq_batch_s* b, hipStream_t st) {
  auto m = std::make_unique<MixedRounds>();
  const size_t budget = ws_budget_bytes();
  size_t total_bytes = 0;
  for (auto& g : b->groups) total_bytes += g.cells.size() * g.plan->workspace_bytes_per_cell();
  int R = (int)std::max<size_t>(1, (total_bytes + budget - 1) / budget);
  std::vector<int> k(b->groups.size());
  for (;; ++R) {
    size_t need = 0;
    for (size_t i = 0; i < b->groups.size(); ++i) {
      k[i] = (int)((b->groups[i].cells.size() + R - 1) / R);
      need += (size_t)k[i] * b->groups[i].plan->workspace_bytes_per_cell();
    }
    if (need <= budget || R >= 1 << 20) break;
  }
  std::vector<size_t> order(b->groups.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return b->groups[x].plan->N > b->groups[y].plan->N; });
  // slots and their workspaces
  std::vector<std::vector<int>> slots_of(b->groups.size());
  for (size_t gi : order)
    for (int j = 0; j < k[gi]; ++j) {
      auto* w = new Workspace();
      m->slot_ws.push_back(w);
      m->slot_group.push_back((int)gi);
      slots_of[gi].push_back((int)m->slot_ws.size() - 1);
      bzq_status s = workspace_init(*w, *b->groups[gi].plan, 1);
      if (s != BZQ_OK) return s;
    }
  // round tables
  int rounds = 0;
  for (size_t gi = 0; gi < b->groups.size(); ++gi)
    rounds = std::max(rounds, (int)((b->groups[gi].cells.size() + k[gi] - 1) / k[gi]));
  m->rounds = rounds;
  m->max_cells = (int)m->slot_ws.size();
  std::vector<MixCell> cells((size_t)rounds * m->max_cells);
  std::vector<int> offs((size_t)rounds * MIX_STAGES * (m->max_cells + 1), 0);
  m->ncells.assign(rounds, 0);
  m->totals.assign(rounds, {});
  for (int r = 0; r < rounds; ++r) {
    int n = 0;
    for (size_t gi : order) {
      const Group& g = b->groups[gi];
      const Plan& p = *g.plan;
      for (int j = 0; j < k[gi]; ++j) {
        const size_t ci = (size_t)r * k[gi] + j;
        if (ci >= g.cells.size()) break;
        const Workspace& w = *m->slot_ws[slots_of[gi][j]];
        MixCell& c = cells[(size_t)r * m->max_cells + n];
        c.N = p.N;
        c.npt = p.npt;
        c.S = p.S;
        c.cell = g.cells[ci];
        c.f = (double2*)b->f[c.cell];
        c.fs = (double2*)w.fs;
        c.q1 = (double2*)w.q1;
        c.q2 = (double2*)w.q2;
        c.fc = w.fc;
        c.fgrid = (float*)w.fgrid;
        c.A = w.A;
        c.B = w.B;
        c.Qpart = (double2*)w.Qpart;
        c.V = (const float*)p.V;
        c.ph = (const double2*)p.ph;
        c.cp = p.cp;
        ++n;
      }
    }
    m->ncells[r] = n;
    for (int stg = 0; stg < MIX_STAGES; ++stg) {
      int* o = &offs[((size_t)r * MIX_STAGES + stg) * (m->max_cells + 1)];
      for (int i = 0; i < n; ++i) {
        const MixCell& c = cells[(size_t)r * m->max_cells + i];
        o[i + 1] = o[i] + mix_items(stg, c.N, c.npt, c.S);
      }
      m->totals[r][stg] = o[n];
    }
  }
  bzq_status s;
  if ((s = m->arena.get(&m->d_cells, cells.size() * sizeof(MixCell))) != BZQ_OK) return s;
  if ((s = m->arena.get(&m->d_offs, offs.size() * sizeof(int))) != BZQ_OK) return s;
  if ((s = m->arena.get(&m->d_outs, b->f.size() * sizeof(double2*))) != BZQ_OK) return s;
  BZQ_HIP_TRY(hipMemcpyAsync(m->d_cells, cells.data(), cells.size() * sizeof(MixCell), hipMemcpyHostToDevice, st));
  BZQ_HIP_TRY(hipMemcpyAsync(m->d_offs, offs.data(), offs.size() * sizeof(int), hipMemcpyHostToDevice, st));
  BZQ_HIP_TRY(hipStreamSynchronize(st));   // the host tables go out of scope
  for (size_t i = 0; i < b->groups.size(); ++i) b->groups[i].cpl = k[i];
  b->mix = std::move(m);
  return BZQ_OK;
}

}  // namespace

extern "C" {

bzq_status bzq_batch_create(bzq_batch* out, const bzq_plan* plans, double* const* f_hats, int count,
                            int cells_per_launch, void* stream) {
  if (!out) return fail(BZQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1 || !plans || !f_hats) return fail(BZQ_EINVAL, "bad batch arguments");
  if (cells_per_launch < -1 || cells_per_launch > kMaxCells)
    return fail(BZQ_EINVAL, "cells_per_launch must lie in [-1, 64]");
  for (int i = 0; i < count; ++i)
    if (!plans[i] || !f_hats[i]) return fail(BZQ_EINVAL, "NULL entry in batch");
  hipStream_t st = (hipStream_t)stream;
  auto* b = new bzq_batch_s();
  b->f.assign(f_hats, f_hats + count);
  std::map<const Plan*, int> gid;
  for (int i = 0; i < count; ++i) {
    auto it = gid.find(plans[i]);
    if (it == gid.end()) {
      gid[plans[i]] = (int)b->groups.size();
      Group g;
      g.plan = plans[i];
      b->groups.push_back(g);
      it = gid.find(plans[i]);
    }
    b->groups[it->second].cells.push_back(i);
  }
  if (cells_per_launch < 0 && !kMixedLaunches) {
    delete b;
    return fail(BZQ_EUNSUPPORTED, "mixed-size launches are switched off: their first run on the device ended in a "
                                  "memory fault whose cause is not known");
  }
  if (kMixedLaunches && cells_per_launch <= 0 && mixed_eligible(b)) {
    bzq_status s = plan_mixed(b, st);
    if (s != BZQ_OK) {
      delete b;
      return s;
    }
    *out = b;
    return BZQ_OK;
  }
  if (cells_per_launch < 0) {
    delete b;
    return fail(BZQ_EUNSUPPORTED, "these plans do not run in mixed-size launches (FP32 table plans with N in "
                                  "{16, 24, 32} and their default kernel variants only)");
  }
  for (auto& g : b->groups) {
    bzq_status s = BZQ_OK;
    if (cells_per_launch > 0)
      g.cpl = std::min<int>(cells_per_launch, (int)g.cells.size());
    else
      s = autotune(g, b->f, st);
    if (s == BZQ_OK) {
      g.ws = new Workspace();
      s = workspace_init(*g.ws, *g.plan, g.cpl);
    }
    if (s != BZQ_OK) {
      delete b;
      return s;
    }
  }
  *out = b;
  return BZQ_OK;
}

bzq_status bzq_batch_collision(bzq_batch b, double* const* Q_hats, void* stream) {
  if (!b || !Q_hats) return fail(BZQ_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  std::vector<double*> q(Q_hats, Q_hats + b->f.size());
  for (double* x : q)
    if (!x) return fail(BZQ_EINVAL, "NULL output in batch");
  for (const auto& g : b->groups)
    for (int c : g.cells)
      if (ranges_overlap(q[c], b->f[c], state_bytes(g.plan->N)))
        return fail(BZQ_EINVAL, "an output overlaps its cell's state");
  if (b->mix) {
    MixedRounds& m = *b->mix;
    m.h_outs = q;
    BZQ_HIP_TRY(hipMemcpyAsync(m.d_outs, m.h_outs.data(), q.size() * sizeof(double*), hipMemcpyHostToDevice, st));
    BZQ_HIP_TRY(hipStreamSynchronize(st));   // h_outs may change with the next call
    return enqueue_mixed(b, false, 0.0, st);
  }
  for (auto& g : b->groups) {
    for (size_t c0 = 0; c0 < g.cells.size(); c0 += g.cpl) {
      const int m = (int)std::min<size_t>(g.cpl, g.cells.size() - c0);
      bzq_status s = enqueue_collision(*g.plan, *g.ws, pack(b->f, g.cells, c0, m), pack(q, g.cells, c0, m), m, st);
      if (s != BZQ_OK) return s;
    }
  }
  return BZQ_OK;
}

bzq_status bzq_batch_step(bzq_batch b, double dt, int n_steps, int use_graph, void* stream) {
  if (!b) return fail(BZQ_EINVAL, "NULL batch");
  if (!std::isfinite(dt) || n_steps < 0) return fail(BZQ_EINVAL, "bad dt or n_steps");
  hipStream_t st = (hipStream_t)stream;
  if (!use_graph) {
    for (int i = 0; i < n_steps; ++i) {
      bzq_status s = enqueue_batch_step(b, dt, st);
      if (s != BZQ_OK) return s;
    }
    return BZQ_OK;
  }
  if (!b->exec || b->graph_dt != dt) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    // record on a private stream (the legacy default stream cannot be
    // captured); nothing runs while recording, the graph is replayed on `st`
    if (!b->capture) BZQ_HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
    std::vector<bool> timing;
    for (auto& g : b->groups) { timing.push_back(g.plan->timing); g.plan->timing = false; }
    BZQ_HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    bzq_status s = enqueue_batch_step(b, dt, b->capture);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->capture, &graph);
    for (size_t i = 0; i < b->groups.size(); ++i) b->groups[i].plan->timing = timing[i];
    if (s != BZQ_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return fail(BZQ_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    b->graph = graph;
    BZQ_HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_dt = dt;
  }
  for (int i = 0; i < n_steps; ++i) BZQ_HIP_TRY(hipGraphLaunch(b->exec, st));
  return BZQ_OK;
}

int bzq_batch_groups(bzq_batch b) { return b ? (int)b->groups.size() : 0; }

bzq_status bzq_batch_group_info(bzq_batch b, int group, int* out) {
  if (!b || !out || group < 0 || group >= (int)b->groups.size()) return fail(BZQ_EINVAL, "bad group");
  const Group& g = b->groups[group];
  out[0] = g.plan->N;
  out[1] = (int)g.cells.size();
  out[2] = g.cpl;
  out[3] = g.tuned ? 1 : 0;
  return BZQ_OK;
}

size_t bzq_batch_device_bytes(bzq_batch b) {
  size_t n = 0;
  if (b) {
    for (auto& g : b->groups) n += g.ws ? g.ws->arena.bytes : 0;
    if (b->mix) {
      for (Workspace* w : b->mix->slot_ws) n += w->arena.bytes;
      n += b->mix->arena.bytes;
    }
  }
  return n;
}

int bzq_batch_rounds(bzq_batch b) { return b && b->mix ? b->mix->rounds : 0; }

bzq_status bzq_batch_destroy(bzq_batch b) {
  if (!b) return BZQ_OK;
  (void)hipDeviceSynchronize();
  delete b;
  return BZQ_OK;
}

bzq_status bzq_collision_batch(const bzq_plan* plans, const double* const* f_hats, double* const* Q_hats,
                               int count, void* stream) {
  if (count < 0 || (count > 0 && (!plans || !f_hats || !Q_hats))) return fail(BZQ_EINVAL, "bad batch arguments");
  for (int i = 0; i < count; ++i) {
    if (!plans[i] || !f_hats[i] || !Q_hats[i]) return fail(BZQ_EINVAL, "NULL entry in batch");
    if (ranges_overlap(f_hats[i], Q_hats[i], state_bytes(plans[i]->N)))
      return fail(BZQ_EINVAL, "f_hat and Q_hat of a cell overlap");
  }
  for (int i = 0; i < count; ++i) {
    bzq_status s = enqueue_collision(*plans[i], plans[i]->ws, single(f_hats[i]), single(Q_hats[i]), 1,
                                     (hipStream_t)stream);
    if (s != BZQ_OK) return s;
  }
  return BZQ_OK;
}

}  // extern "C"
