// pa_stepper.cpp -- continuous batching: one temperature step for an arbitrary
// set of resident instances in one set of launches.
//
// Method: Amey & Machta, arXiv:1711.02146 (Sec. II loop: resample with
// Eqs. 1-2, then sweeps at the new temperature; Eq. 9 free energy; Sec. III.A
// rho_t; Sec. III.C culling fraction).
//
// Unlike a batch (one schedule, one captured graph replayed), the set of
// instances, their inverse temperatures and their sweep counts may change
// from call to call, so requests can join and leave between steps.  Each call
// writes the set's descriptors, per-instance step parameters and exp rows
// into the stepper's workspace with one host-to-device copy, then launches,
// for every instance of the set at once:
//   zero accumulators -> histogram (current population) -> FP64 table
//   -> counts -> scan -> scatter -> fused copy + sweeps (one launch per
//   (layout, L)) -> zero accumulators -> histogram -> family sums -> record,
// and reads the records back.  The arithmetic and the random numbers are
// those of pa_resample + pa_sweep + pa_observables on each instance alone.
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

struct StepperLayout {
  size_t off_pops, off_steps, off_rec, off_ctr, off_u32, off_E, total;
  size_t n_u32, e_doubles;
};

bool stepper_layout(uint32_t max_pops, uint32_t max_L, StepperLayout* out) {
  if (max_pops == 0 || max_pops > (1u << 20) || max_L < 4 || max_L > (uint32_t)pa::kMaxL)
    return false;
  StepperLayout l{};
  const size_t N = (size_t)max_L * max_L * max_L;
  // groups: per-pop, slots and histogram (n ids + n + 1 starts each), sweep
  // groups (n ids + one start per group + n; at most 14 (layout, L) kinds)
  l.n_u32 = 3 * (2 * (size_t)max_pops + 1) + (2 * (size_t)max_pops + 16);
  l.e_doubles = (size_t)max_pops * (3 * N + 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  l.off_pops = take((size_t)max_pops * sizeof(pa::DevPop));
  l.off_steps = take((size_t)max_pops * sizeof(pa::PopStep));
  l.off_rec = take((size_t)max_pops * sizeof(pa::StepRecord));
  l.off_ctr = take(4);
  l.off_u32 = take(l.n_u32 * 4);
  l.off_E = take(l.e_doubles * 8);  // last: only the used part is copied
  l.total = o;
  *out = l;
  return true;
}

}  // namespace

struct pa_stepper {
  uint32_t max_pops = 0, max_L = 0;
  hipStream_t stream = nullptr;
  uint8_t* ws = nullptr;
  StepperLayout lay{};
  uint8_t* h_img = nullptr;         // pinned host image of the workspace prefix
  pa::StepRecord* h_rec = nullptr;  // pinned records
  bool failed = false;
};

extern "C" {

size_t pa_stepper_workspace_bytes(uint32_t max_pops, uint32_t max_L) {
  StepperLayout l;
  if (!stepper_layout(max_pops, max_L, &l)) return 0;
  return l.total;
}

int pa_stepper_create(uint32_t max_pops, uint32_t max_L, void* d_workspace, size_t ws_bytes,
                      void* hip_stream, pa_stepper** out) {
  if (!out) return PA_EINVAL;
  *out = nullptr;
  StepperLayout l;
  if (!stepper_layout(max_pops, max_L, &l) || !d_workspace) return PA_EINVAL;
  if (ws_bytes < l.total) return PA_ENOMEM;
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) return PA_EINVAL;
  pa_stepper* s = new (std::nothrow) pa_stepper();
  if (!s) return PA_EINVAL;
  s->max_pops = max_pops;
  s->max_L = max_L;
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->ws = static_cast<uint8_t*>(d_workspace);
  s->lay = l;
  if (hipHostMalloc(reinterpret_cast<void**>(&s->h_img), l.total) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->h_rec), (size_t)max_pops * sizeof(pa::StepRecord)) !=
          hipSuccess) {
    pa_stepper_free(s);
    return PA_EDEVICE;
  }
  *out = s;
  return PA_OK;
}

int pa_stepper_free(pa_stepper* s) {
  if (!s) return PA_EINVAL;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->h_img) (void)hipHostFree(s->h_img);
  if (s->h_rec) (void)hipHostFree(s->h_rec);
  delete s;
  return PA_OK;
}

int pa_stepper_step(pa_stepper* s, pa_instance* const* pops, uint32_t n, const double* beta_next,
                    const uint32_t* n_sweeps, pa_obs* obs, int32_t* status) {
  if (!s || s->failed) return PA_ESTATE;
  if (n == 0) return PA_OK;
  if (!pops || !beta_next || !n_sweeps || n > s->max_pops) return PA_EINVAL;
  for (uint32_t p = 0; p < n; ++p) {
    pa_instance* in = pops[p];
    if (!in) return PA_EINVAL;
    if (in->failed || in->in_batch || in->pending_gather) return PA_ESTATE;
    if (in->stream != s->stream || in->dev.L > s->max_L) return PA_EINVAL;
    if (in->dev.model != pa::kModelPm) return PA_EINVAL;  // exp rows cover U levels only
    if (!std::isfinite(beta_next[p])) return PA_EINVAL;
    if (in->sweeps + n_sweeps[p] > 0xFFFFFFFFull) return PA_EINVAL;  // 32-bit sweep counter
    for (uint32_t q = 0; q < p; ++q)
      if (pops[q] == in) return PA_EINVAL;
  }
  // every instance of the set counts one call (fault injection); one that
  // fails fails the whole call before anything is queued
  for (uint32_t p = 0; p < n; ++p) {
    const int rc = pa_host::count_call(pops[p]);
    if (rc != PA_OK) {
      if (status) status[p] = rc;
      return rc;
    }
  }
  const StepperLayout& l = s->lay;
  uint8_t* const img = s->h_img;
  uint8_t* const w = s->ws;
  pa::DevPop* dpops = reinterpret_cast<pa::DevPop*>(img + l.off_pops);
  pa::PopStep* steps = reinterpret_cast<pa::PopStep*>(img + l.off_steps);
  std::memset(img + l.off_rec, 0, (size_t)n * sizeof(pa::StepRecord));
  *reinterpret_cast<uint32_t*>(img + l.off_ctr) = 0;
  double* E = reinterpret_cast<double*>(img + l.off_E);
  const double* dE = reinterpret_cast<const double*>(w + l.off_E);
  size_t e_used = 0;
  uint32_t max_levels = 0;
  for (uint32_t p = 0; p < n; ++p) {
    const pa_instance* in = pops[p];
    dpops[p] = in->dev;
    max_levels = std::max(max_levels, in->dev.n_levels);
    // exp row of this instance's step: E[d] = exp(-dbeta 2d), the host table's weight
    const double dbeta = beta_next[p] - in->beta;
    double* row = E + e_used;
    for (uint32_t d = 0; d < in->dev.n_levels; ++d) row[d] = std::exp(-dbeta * (double)(2 * (int64_t)d));
    pa::PopStep& ps = steps[p];
    ps = pa::PopStep{};
    pa_host::thresholds(beta_next[p], ps.thr);
    ps.erow = dE + e_used;
    ps.t0 = (uint32_t)in->sweeps;
    ps.n_sweeps = n_sweeps[p];
    ps.gather = 1;
    ps.cur = in->cur;
    ps.step = in->step + 1;
    ps.flags = pa::kStepSticky;
    e_used += in->dev.n_levels;
  }
  pa_host::GroupTables gt;
  gt.d_base = reinterpret_cast<uint32_t*>(w + l.off_u32);
  std::vector<uint32_t> all(n), one(n, 1), slots(n), hist(n);
  for (uint32_t p = 0; p < n; ++p) {
    all[p] = p;
    slots[p] = pa::blocks_slots(pops[p]->dev.capacity);
    hist[p] = pa::blocks_hist(pops[p]->dev.capacity);
  }
  const pa::Group g_perpop = gt.add(all, one);
  const pa::Group g_slots = gt.add(all, slots);
  const pa::Group g_hist = gt.add(all, hist);
  struct SweepGroup {
    uint32_t layout, L;
    uint32_t split;  // waves per tile
    pa::Group g;
  };
  std::vector<SweepGroup> g_sweep;
  std::map<std::pair<uint32_t, uint32_t>, std::vector<uint32_t>> by_kind;
  for (uint32_t p = 0; p < n; ++p) by_kind[{pops[p]->dev.layout, pops[p]->dev.L}].push_back(p);
  for (const auto& kv : by_kind) {
    uint64_t tiles = 0;
    for (uint32_t p : kv.second) tiles += (pops[p]->dev.R + 63) / 64;
    const uint32_t split =
        pa::sweep_split_for(pa::kModelPm, kv.first.first, kv.first.second, tiles);
    std::vector<uint32_t> nb;
    for (uint32_t p : kv.second) nb.push_back(pa::blocks_sweep(pops[p]->dev.capacity));
    g_sweep.push_back({kv.first.first, kv.first.second, split, gt.add(kv.second, nb)});
  }
  if (gt.u32.size() > l.n_u32) return PA_EINVAL;
  std::memcpy(img + l.off_u32, gt.u32.data(), gt.u32.size() * 4);

  pa::BatchDev B{};
  B.pops = reinterpret_cast<const pa::DevPop*>(w + l.off_pops);
  B.steps = reinterpret_cast<const pa::PopStep*>(w + l.off_steps);
  B.step_ctr = reinterpret_cast<const uint32_t*>(w + l.off_ctr);
  B.records = reinterpret_cast<pa::StepRecord*>(w + l.off_rec);
  B.n_pops = n;

  hipStream_t st = s->stream;
  auto dev_fail = [&]() {
    s->failed = true;
    return PA_EDEVICE;
  };
  const size_t bytes = l.off_E + e_used * 8;
  if (hipMemcpyAsync(w, img, bytes, hipMemcpyHostToDevice, st) != hipSuccess) return dev_fail();
  bool ok = pa::launch_zero_acc(B, g_perpop, st) == hipSuccess &&
            pa::launch_hist(B, g_hist, max_levels, false, st) == hipSuccess &&
            pa::launch_table(B, g_perpop, st) == hipSuccess &&
            pa::launch_counts(B, g_slots, st) == hipSuccess &&
            pa::launch_scan(B, g_perpop, st) == hipSuccess &&
            pa::launch_scatter(B, g_slots, st) == hipSuccess;
  for (const auto& sg : g_sweep) ok = ok && pa::launch_sweep(B, sg.g, sg.layout, sg.L, sg.split, pa::kModelPm, st) ==
                                             hipSuccess;
  ok = ok && pa::launch_zero_acc(B, g_perpop, st) == hipSuccess &&
       pa::launch_hist(B, g_hist, max_levels, true, st) == hipSuccess &&
       pa::launch_family(B, g_slots, true, st) == hipSuccess &&
       pa::launch_record(B, g_perpop, st) == hipSuccess;
  if (!ok) return dev_fail();
  if (hipMemcpyAsync(s->h_rec, w + l.off_rec, (size_t)n * sizeof(pa::StepRecord),
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return dev_fail();

  for (uint32_t p = 0; p < n; ++p) {
    pa_instance* in = pops[p];
    const pa::DevPop& P = in->dev;
    const pa::StepRecord& r = s->h_rec[p];
    pa_obs* o = obs ? obs + p : nullptr;
    if (o) std::memset(o, 0, sizeof(*o));
    if (r.status == 2) {
      // the sweep kernel found its LDS layout unusable and wrote nothing
      if (status) status[p] = PA_EDEVICE;
      in->failed = true;
      s->failed = true;
      continue;
    }
    if (r.status != 0) {
      // the copy step would overflow the capacity: nothing after the scan ran
      // for this instance, so its population is as it was; clear its flags
      if (status) status[p] = PA_ECAPACITY;
      pa::DevScalars sc{};
      if (hipMemcpy(&sc, P.sc, sizeof(sc), hipMemcpyDeviceToHost) != hipSuccess) return dev_fail();
      sc.dead = 0;
      sc.err = 0;
      if (hipMemcpy(P.sc, &sc, sizeof(sc), hipMemcpyHostToDevice) != hipSuccess) return dev_fail();
      continue;
    }
    if (status) status[p] = PA_OK;
    const double dbeta = beta_next[p] - in->beta;
    const double lnQ = std::log(r.S) - std::log((double)r.R_old) -
                       dbeta * (double)(2 * r.jmin - 3 * (int)P.N);
    in->sum_lnQ = in->sum_lnQ + lnQ;
    in->beta = beta_next[p];
    in->step += 1;
    in->sweeps += n_sweeps[p];
    in->cur ^= 1u;
    in->R_tilde = r.R_new;
    in->last_dbeta = dbeta;
    in->last_lnQ = lnQ;
    in->last_eps = r.eps;
    in->last_n_culled = r.n_culled;
    in->last_R_old = r.R_old;
    in->hist_valid = false;
    if (o) {
      o->beta = in->beta;
      o->dbeta = dbeta;
      o->lnQ = lnQ;
      o->beta_F = -((double)P.N * std::log(2.0) + in->sum_lnQ);
      o->mean_E = r.R_new ? (double)r.sumE / (double)r.R_new : 0.0;
      o->sum_eta2 = r.sum_eta2;
      o->rho_t = (double)r.sum_eta2 / (double)P.R;
      o->eps_expected = r.eps;
      o->R_tilde = r.R_new;
      o->n_culled = r.n_culled;
      o->E_min = r.E_min;
      o->E_lowest = (double)r.E_min;
      o->n_at_E_min = r.n_at_E_min;
      o->step = in->step;
      o->sweeps_done = in->sweeps;
      o->sum_lnQ = in->sum_lnQ;
    }
  }
  return s->failed ? PA_EDEVICE : PA_OK;
}

}  // extern "C"
