// pa_batch.cpp -- the batch engine of libpa: many populations advanced
// through one temperature schedule with one captured HIP graph per step.
//
// Method: Amey & Machta, arXiv:1711.02146 (Sec. II loop: resample with
// Eqs. 1-2, then sweeps; Eq. 9 free energy; Sec. III.A rho_t; Sec. III.C
// culling fraction).
//
// A step of the graph, for every population of the batch:
//   table (device FP64; exp row of the step from the host)  -> counts -> scan
//   -> scatter -> sweep (one launch per (layout, L) group, fused copy)
//   -> zero accumulators -> histogram -> family sums -> record -> overlaps
//   -> advance the device step counter.
// The per-step parameters of every population are laid out in device memory
// at creation and indexed by the step counter, so the same graph is replayed
// for every step.  The host finishes ln Q = ln S - ln R~ - dbeta E_min with
// its own log, exactly as the single-instance path does, so the scalars match
// that path bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/pa.h"
#include "pa_host_state.hpp"
#include "pa_internal.hpp"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct BatchLayout {
  size_t off_pops, off_steps, off_rec, off_q, off_E, off_ctr, off_u32, total;
  size_t e_stride;  // doubles per exp row
  size_t n_u32;
};

bool batch_layout(uint32_t n_pops, uint32_t n_pairs, uint32_t n_steps, uint32_t max_L,
                  BatchLayout* out) {
  if (n_pops == 0 || n_steps == 0 || max_L < 4 || max_L > (uint32_t)pa::kMaxL) return false;
  if ((uint64_t)n_pops * n_steps > (1ull << 28)) return false;
  BatchLayout l{};
  const uint64_t N = (uint64_t)max_L * max_L * max_L;
  l.e_stride = (size_t)(3 * N + 1);
  // group tables: 3 groups of (n pop ids + n + 1 starts), sweep groups
  // (n ids + n + 16 starts), pair groups (n_pairs ids + n_pairs + 2 starts)
  // and the 2 n_pairs pair members
  l.n_u32 = 3 * (2 * (size_t)n_pops + 1) + (2 * (size_t)n_pops + 16) + 4 * (size_t)n_pairs + 2;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  l.off_pops = take((size_t)n_pops * sizeof(pa::DevPop));
  l.off_steps = take((size_t)n_steps * n_pops * sizeof(pa::PopStep));
  l.off_rec = take((size_t)n_steps * n_pops * sizeof(pa::StepRecord));
  l.off_q = take((size_t)n_steps * n_pairs * 65 * 8);
  l.off_E = take((size_t)n_steps * l.e_stride * 8);
  l.off_ctr = take(4);
  l.off_u32 = take(l.n_u32 * 4);
  l.total = o;
  *out = l;
  return true;
}

}  // namespace

struct pa_batch {
  std::vector<pa_instance*> pops;
  std::vector<uint32_t> pairs;
  std::vector<double> betas;
  uint32_t n_pops = 0, n_pairs = 0, n_steps = 0, n_sweeps = 0, done = 0;
  hipStream_t stream = nullptr;
  uint8_t* ws = nullptr;
  BatchLayout lay{};
  pa::BatchDev dev{};
  uint32_t* d_ctr = nullptr;
  pa::Group g_perpop{}, g_slots{}, g_hist{};
  struct SweepGroup {
    uint32_t layout, L;
    uint32_t split;  // waves per tile
    pa::Group g;
  };
  std::vector<SweepGroup> g_sweep;
  struct PairGroup {
    uint32_t layout;
    pa::Group g;
  };
  std::vector<PairGroup> g_pairs;  // one overlap launch per spin layout
  const uint32_t* d_pair_pops = nullptr;
  uint32_t max_levels = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // starting point of every population
  std::vector<uint32_t> cur0, step0;
  std::vector<uint64_t> sweeps0;
  std::vector<double> sum_lnQ0;
  bool failed = false;
  bool finished = false;  // results fetched: the instances are released
};

namespace {

#define PB_HIP(call)                   \
  do {                                 \
    if ((call) != hipSuccess) {        \
      b->failed = true;                \
      return PA_EDEVICE;               \
    }                                  \
  } while (0)

// Steps of the schedule recorded in the graph.
int capture_step(pa_batch* b) {
  const pa::BatchDev& B = b->dev;
  hipStream_t s = b->stream;
  PB_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  bool ok = pa::launch_table(B, b->g_perpop, s) == hipSuccess &&
            pa::launch_counts(B, b->g_slots, s) == hipSuccess &&
            pa::launch_scan(B, b->g_perpop, s) == hipSuccess &&
            pa::launch_scatter(B, b->g_slots, s) == hipSuccess;
  for (const auto& sg : b->g_sweep)
    ok = ok && pa::launch_sweep(B, sg.g, sg.layout, sg.L, sg.split, pa::kModelPm, s) == hipSuccess;
  ok = ok && pa::launch_zero_acc(B, b->g_perpop, s) == hipSuccess &&
       pa::launch_hist(B, b->g_hist, b->max_levels, true, s) == hipSuccess &&
       pa::launch_family(B, b->g_slots, true, s) == hipSuccess &&
       pa::launch_record(B, b->g_perpop, s) == hipSuccess;
  for (const auto& pg : b->g_pairs)
    ok = ok && pa::launch_overlap(B, pg.g, b->d_pair_pops, pg.layout, true, 0, 0, s) == hipSuccess;
  ok = ok && pa::launch_advance(b->d_ctr, s) == hipSuccess;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (!ok || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    b->failed = true;
    return PA_EDEVICE;
  }
  b->graph = g;
  PB_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  return PA_OK;
}

}  // namespace

extern "C" {

size_t pa_batch_workspace_bytes(uint32_t n_pops, uint32_t n_pairs, uint32_t n_steps,
                                uint32_t max_L) {
  BatchLayout l;
  if (!batch_layout(n_pops, n_pairs, n_steps, max_L, &l)) return 0;
  return l.total;
}

int pa_batch_create(pa_instance* const* pops, uint32_t n_pops, const uint32_t* pairs,
                    uint32_t n_pairs, const double* betas, uint32_t n_steps, uint32_t n_sweeps,
                    void* d_workspace, size_t ws_bytes, pa_batch** out) {
  if (!out || !pops || !betas || !d_workspace || n_pops == 0 || n_steps == 0) return PA_EINVAL;
  *out = nullptr;
  // the step graph is captured from the instances' stream: it must be a
  // created stream, not the legacy default stream
  if (!pops[0] || !pops[0]->stream) return PA_EINVAL;
  if (n_pairs && !pairs) return PA_EINVAL;
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) return PA_EINVAL;
  uint32_t max_L = 0;
  for (uint32_t p = 0; p < n_pops; ++p) {
    pa_instance* in = pops[p];
    if (!in || in->failed || in->in_batch || in->pending_gather) return PA_ESTATE;
    if (in->stream != pops[0]->stream) return PA_EINVAL;
    if (in->dev.model != pa::kModelPm) return PA_EINVAL;  // per-step exp rows cover U levels
    if (in->beta != betas[0]) return PA_EINVAL;
    for (uint32_t q = 0; q < p; ++q)
      if (pops[q] == in) return PA_EINVAL;
    max_L = std::max(max_L, in->dev.L);
    if (in->sweeps + (uint64_t)n_steps * n_sweeps > 0xFFFFFFFFull) return PA_EINVAL;
  }
  for (uint32_t s = 0; s <= n_steps; ++s)
    if (!std::isfinite(betas[s])) return PA_EINVAL;
  for (uint32_t k = 0; k < n_pairs; ++k) {
    const uint32_t a = pairs[2 * k], c = pairs[2 * k + 1];
    if (a >= n_pops || c >= n_pops || a == c) return PA_EINVAL;
    if (pops[a]->dev.L != pops[c]->dev.L || pops[a]->dev.layout != pops[c]->dev.layout)
      return PA_EINVAL;
  }
  BatchLayout l;
  if (!batch_layout(n_pops, n_pairs, n_steps, max_L, &l)) return PA_EINVAL;
  if (ws_bytes < l.total) return PA_ENOMEM;

  pa_batch* b = new (std::nothrow) pa_batch();
  if (!b) return PA_EINVAL;
  b->pops.assign(pops, pops + n_pops);
  if (n_pairs) b->pairs.assign(pairs, pairs + 2 * n_pairs);
  b->betas.assign(betas, betas + n_steps + 1);
  b->n_pops = n_pops;
  b->n_pairs = n_pairs;
  b->n_steps = n_steps;
  b->n_sweeps = n_sweeps;
  b->stream = pops[0]->stream;
  b->ws = static_cast<uint8_t*>(d_workspace);
  b->lay = l;
  uint8_t* w = b->ws;

  // --- host images of everything the graph reads --------------------------
  std::vector<pa::DevPop> dpops(n_pops);
  for (uint32_t p = 0; p < n_pops; ++p) {
    dpops[p] = pops[p]->dev;
    b->max_levels = std::max(b->max_levels, pops[p]->dev.n_levels);
    b->cur0.push_back(pops[p]->cur);
    b->step0.push_back(pops[p]->step);
    b->sweeps0.push_back(pops[p]->sweeps);
    b->sum_lnQ0.push_back(pops[p]->sum_lnQ);
  }
  // exp rows: E_s[d] = exp(-dbeta_s * 2d), the host table's weight for j - j_min = d
  std::vector<double> E((size_t)n_steps * l.e_stride);
  for (uint32_t s = 1; s <= n_steps; ++s) {
    const double dbeta = betas[s] - betas[s - 1];
    double* row = E.data() + (size_t)(s - 1) * l.e_stride;
    for (size_t d = 0; d < l.e_stride; ++d) row[d] = std::exp(-dbeta * (double)(2 * (int64_t)d));
  }
  const double* dE = reinterpret_cast<const double*>(w + l.off_E);
  std::vector<pa::PopStep> steps((size_t)n_steps * n_pops);
  for (uint32_t s = 0; s < n_steps; ++s) {
    unsigned long long thr[3];
    pa_host::thresholds(betas[s + 1], thr);
    for (uint32_t p = 0; p < n_pops; ++p) {
      pa::PopStep& ps = steps[(size_t)s * n_pops + p];
      ps = pa::PopStep{};
      ps.thr[0] = thr[0];
      ps.thr[1] = thr[1];
      ps.thr[2] = thr[2];
      ps.erow = dE + (size_t)s * l.e_stride;
      ps.t0 = (uint32_t)(b->sweeps0[p] + (uint64_t)s * n_sweeps);
      ps.n_sweeps = n_sweeps;
      ps.gather = 1;
      ps.cur = b->cur0[p] ^ (s & 1u);
      ps.step = b->step0[p] + s + 1;
      ps.flags = pa::kStepSticky;
    }
  }
  // group tables
  pa_host::GroupTables gt;
  gt.d_base = reinterpret_cast<uint32_t*>(w + l.off_u32);
  gt.u32.reserve(l.n_u32);
  auto add_group = [&](const std::vector<uint32_t>& members, const std::vector<uint32_t>& blocks) {
    return gt.add(members, blocks);
  };
  std::vector<uint32_t>& u32 = gt.u32;
  uint32_t* const d_u32 = gt.d_base;
  std::vector<uint32_t> all(n_pops), one(n_pops, 1), slots(n_pops), hist(n_pops);
  for (uint32_t p = 0; p < n_pops; ++p) {
    all[p] = p;
    slots[p] = pa::blocks_slots(pops[p]->dev.capacity);
    hist[p] = pa::blocks_hist(pops[p]->dev.capacity);
  }
  b->g_perpop = add_group(all, one);
  b->g_slots = add_group(all, slots);
  b->g_hist = add_group(all, hist);
  std::map<std::pair<uint32_t, uint32_t>, std::vector<uint32_t>> by_kind;
  for (uint32_t p = 0; p < n_pops; ++p) by_kind[{pops[p]->dev.layout, pops[p]->dev.L}].push_back(p);
  for (const auto& kv : by_kind) {
    uint64_t tiles = 0;
    for (uint32_t p : kv.second) tiles += (pops[p]->dev.R + 63) / 64;
    const uint32_t split =
        pa::sweep_split_for(pa::kModelPm, kv.first.first, kv.first.second, tiles);
    std::vector<uint32_t> nb;
    for (uint32_t p : kv.second) nb.push_back(pa::blocks_sweep(pops[p]->dev.capacity));
    b->g_sweep.push_back({kv.first.first, kv.first.second, split, add_group(kv.second, nb)});
  }
  for (uint32_t layout : {(uint32_t)PA_LAYOUT_INT8, (uint32_t)PA_LAYOUT_BITPACK64}) {
    std::vector<uint32_t> ids, nb;
    for (uint32_t k = 0; k < n_pairs; ++k) {
      if (pops[pairs[2 * k]]->dev.layout != layout) continue;
      ids.push_back(k);
      nb.push_back(std::min(pops[pairs[2 * k]]->dev.capacity,
                            pops[pairs[2 * k + 1]]->dev.capacity) / 64);
    }
    if (!ids.empty()) b->g_pairs.push_back({layout, add_group(ids, nb)});
  }
  b->d_pair_pops = d_u32 + u32.size();
  for (uint32_t k = 0; k < 2 * n_pairs; ++k) u32.push_back(pairs[k]);
  if (u32.size() > l.n_u32) {
    delete b;
    return PA_EINVAL;
  }

  pa::BatchDev& B = b->dev;
  B.pops = reinterpret_cast<const pa::DevPop*>(w + l.off_pops);
  B.steps = reinterpret_cast<const pa::PopStep*>(w + l.off_steps);
  b->d_ctr = reinterpret_cast<uint32_t*>(w + l.off_ctr);
  B.step_ctr = b->d_ctr;
  B.records = reinterpret_cast<pa::StepRecord*>(w + l.off_rec);
  B.qhist = n_pairs ? reinterpret_cast<unsigned long long*>(w + l.off_q) : nullptr;
  B.n_pops = n_pops;
  B.n_pairs = n_pairs;

  hipStream_t s = b->stream;
  auto fail = [&](int rc) {
    pa_batch_free(b);
    return rc;
  };
  const uint32_t zero = 0;
  if (hipMemcpyAsync(w + l.off_pops, dpops.data(), dpops.size() * sizeof(pa::DevPop),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(w + l.off_steps, steps.data(), steps.size() * sizeof(pa::PopStep),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(w + l.off_E, E.data(), E.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(w + l.off_u32, u32.data(), u32.size() * 4, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(b->d_ctr, &zero, 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      pa::launch_fill_u32(reinterpret_cast<uint32_t*>(w + l.off_rec), 0u,
                          (size_t)n_steps * n_pops * sizeof(pa::StepRecord) / 4, s) != hipSuccess ||
      (n_pairs && pa::launch_fill_u32(reinterpret_cast<uint32_t*>(w + l.off_q), 0u,
                                      (size_t)n_steps * n_pairs * 65 * 2, s) != hipSuccess))
    return fail(PA_EDEVICE);
  // clear the per-population failure flags, then the histogram of the
  // starting populations (the first step's table reads it)
  for (uint32_t p = 0; p < n_pops; ++p) {
    if (pa::launch_fill_u32(&pops[p]->dev.sc->dead, 0u, 1, s) != hipSuccess)
      return fail(PA_EDEVICE);
  }
  if (pa::launch_zero_acc(B, b->g_perpop, s) != hipSuccess ||
      pa::launch_hist(B, b->g_hist, b->max_levels, false, s) != hipSuccess)
    return fail(PA_EDEVICE);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(PA_EDEVICE);
  const int rc = capture_step(b);
  if (rc) return fail(rc);
  for (uint32_t p = 0; p < n_pops; ++p) pops[p]->in_batch = true;
  *out = b;
  return PA_OK;
}

int pa_batch_run(pa_batch* b, uint32_t n_steps) {
  if (!b || b->failed || b->finished) return PA_ESTATE;
  if (n_steps > b->n_steps - b->done) return PA_EINVAL;
  for (uint32_t k = 0; k < n_steps; ++k) PB_HIP(hipGraphLaunch(b->exec, b->stream));
  b->done += n_steps;
  return PA_OK;
}

int pa_batch_results(pa_batch* b, pa_obs* obs, uint64_t* qhist, int32_t* status,
                     uint32_t* steps_done) {
  if (!b || b->failed || b->finished) return PA_ESTATE;
  PB_HIP(hipStreamSynchronize(b->stream));
  const uint32_t n = b->done, np = b->n_pops;
  std::vector<pa::StepRecord> rec((size_t)n * np);
  if (n) {
    PB_HIP(hipMemcpy(rec.data(), b->ws + b->lay.off_rec, rec.size() * sizeof(pa::StepRecord),
                     hipMemcpyDeviceToHost));
    if (qhist && b->n_pairs)
      PB_HIP(hipMemcpy(qhist, b->ws + b->lay.off_q, (size_t)n * b->n_pairs * 65 * 8,
                       hipMemcpyDeviceToHost));
  }
  if (steps_done) *steps_done = n;
  for (uint32_t p = 0; p < np; ++p) {
    pa_instance* in = b->pops[p];
    const pa::DevPop& P = in->dev;
    double sum_lnQ = b->sum_lnQ0[p];
    uint32_t completed = 0;
    int32_t st = PA_OK;
    for (uint32_t s = 0; s < n; ++s) {
      const pa::StepRecord& r = rec[(size_t)s * np + p];
      pa_obs* o = obs ? obs + (size_t)s * np + p : nullptr;
      if (r.status != 0) {
        st = r.status == 2 ? PA_EDEVICE : PA_ECAPACITY;
        if (o) std::memset(o, 0, sizeof(*o));
        for (uint32_t t = s + 1; t < n; ++t)
          if (obs) std::memset(obs + (size_t)t * np + p, 0, sizeof(pa_obs));
        break;
      }
      const double dbeta = b->betas[s + 1] - b->betas[s];
      const double lnQ = std::log(r.S) - std::log((double)r.R_old) -
                         dbeta * (double)(2 * r.jmin - 3 * (int)P.N);
      sum_lnQ = sum_lnQ + lnQ;
      if (o) {
        std::memset(o, 0, sizeof(*o));
        o->beta = b->betas[s + 1];
        o->dbeta = dbeta;
        o->lnQ = lnQ;
        o->beta_F = -((double)P.N * std::log(2.0) + sum_lnQ);
        o->mean_E = r.R_new ? (double)r.sumE / (double)r.R_new : 0.0;
        o->sum_eta2 = r.sum_eta2;
        o->rho_t = (double)r.sum_eta2 / (double)P.R;
        o->eps_expected = r.eps;
        o->R_tilde = r.R_new;
        o->n_culled = r.n_culled;
        o->E_min = r.E_min;
        o->E_lowest = (double)r.E_min;
      o->n_at_E_min = r.n_at_E_min;
        o->step = b->step0[p] + s + 1;
        o->sweeps_done = b->sweeps0[p] + (uint64_t)(s + 1) * b->n_sweeps;
        o->sum_lnQ = sum_lnQ;
      }
      completed = s + 1;
      in->last_dbeta = dbeta;
      in->last_lnQ = lnQ;
      in->last_eps = r.eps;
      in->last_n_culled = r.n_culled;
      in->last_R_old = r.R_old;
      in->R_tilde = r.R_new;
    }
    if (status) status[p] = st;
    // the instance continues from its last completed step
    in->beta = b->betas[completed];
    in->step = b->step0[p] + completed;
    in->sweeps = b->sweeps0[p] + (uint64_t)completed * b->n_sweeps;
    in->cur = b->cur0[p] ^ (completed & 1u);
    in->sum_lnQ = sum_lnQ;
    in->pending_gather = false;
    in->hist_valid = false;
    if (st == PA_EDEVICE) {
      in->failed = true;  // the sweep kernel found its LDS layout unusable
    } else if (st != PA_OK) {
      // the failed step left the population as it was; clear its flags
      pa::DevScalars sc{};
      PB_HIP(hipMemcpy(&sc, P.sc, sizeof(sc), hipMemcpyDeviceToHost));
      sc.dead = 0;
      sc.err = 0;
      PB_HIP(hipMemcpy(P.sc, &sc, sizeof(sc), hipMemcpyHostToDevice));
    }
    in->in_batch = false;  // the instance is its own again
  }
  b->finished = true;
  return PA_OK;
}

int pa_batch_free(pa_batch* b) {
  if (!b) return PA_EINVAL;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (pa_instance* in : b->pops)
    if (in) in->in_batch = false;
  delete b;
  return PA_OK;
}

}  // extern "C"
