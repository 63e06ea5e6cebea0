// pa_host_state.hpp -- host-side state of libpa instances, shared by the
// single-instance C ABI (pa_host.cpp) and the batch engine (pa_batch.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/pa.h"
#include "pa_internal.hpp"

namespace pa_host {

using pa::DevPop;
using pa::DevScalars;
using pa::SiteEntry;

// Group tables of calls on one instance (two-entry start arrays {0, blocks}).
struct MetaU32 {
  uint32_t pop0[2];       // {0, 1}: member populations of a one-population set (+ partner)
  uint32_t perpop[2];     // one workgroup
  uint32_t slots[2];      // capacity / 256 workgroups
  uint32_t hist[2];       // histogram workgroups
  uint32_t tiles[2];      // sweep workgroups
  uint32_t etiles[2];     // one-wave tiles (energy recompute)
  uint32_t pair_pops[2];  // {0, 1}: the instance and its overlap partner
  uint32_t pairs[2];      // overlap workgroups, set per call
  uint32_t rsum[2];       // PA_MODEL_GAUSS weight reductions: min(capacity / 256, kRealSumBlocks)
};

struct Layout {
  uint32_t L, N, R, cap_limit, capacity, layout, n_levels, n_blocks, model, rowk_stride;
  size_t spins_bytes;
  size_t hist_bytes;  // the histogram's share of its block (n_levels words, 64-byte multiple)
  size_t off_spins[2], off_U[2], off_fam[2], off_counts, off_offsets, off_src, off_bsum, off_boff,
      off_bcull, off_hist, off_table, off_sites, off_psites, off_cm, off_rowj, off_rowk, off_gthr, off_ovl,
      off_lovl, off_lpart, off_sc, off_rs, off_pops, off_meta, off_rhe, off_rthr, off_rthr32, off_rpart, off_gaddr;
  size_t total;
};

// Host image of the group tables of a multi-population launch set: each
// group is (member population ids, n + 1 workgroup starts), laid out in one
// u32 array that is copied to d_base.
struct GroupTables {
  std::vector<uint32_t> u32;
  uint32_t* d_base = nullptr;

  pa::Group add(const std::vector<uint32_t>& members, const std::vector<uint32_t>& blocks) {
    pa::Group g{};
    g.n = (uint32_t)members.size();
    g.pop = d_base + u32.size();
    for (uint32_t m : members) u32.push_back(m);
    g.start = d_base + u32.size();
    uint32_t acc = 0;
    u32.push_back(0);
    for (uint32_t nb : blocks) {
      acc += nb;
      u32.push_back(acc);
    }
    g.blocks = acc;
    return g;
  }
};

// Metropolis thresholds: accept dE > 0 iff word < floor(2^32 exp(-beta dE)).
inline void thresholds(double beta, unsigned long long thr[3]) {
  for (int i = 0; i < 3; ++i) {
    const double dE = (double)(4 * (i + 1));
    thr[i] = (unsigned long long)std::floor(std::ldexp(std::exp(-beta * dE), 32));
  }
}

}  // namespace pa_host

struct pa_instance {
  pa_host::Layout lay;
  pa::DevPop dev;
  pa::DevPop* d_pops = nullptr;      // device copy of dev (slot 0) and an overlap partner (slot 1)
  pa_host::MetaU32* d_meta = nullptr;
  pa_host::MetaU32 meta{};
  hipStream_t stream = nullptr;
  uint8_t* ws = nullptr;
  std::vector<pa::SiteEntry> sites;
  std::vector<uint16_t> cm_of_site;
  std::vector<uint64_t> rowj;
  std::vector<int8_t> rowk;          // PA_MODEL_GAUSS16 row couplings
  // PA_MODEL_GAUSS16: energy window of the histogram in h_hist (valid with hist_valid)
  int32_t E_lo = 0;
  uint32_t n_win = 0;
  // host mirror of the population state
  uint32_t cur = 0;
  uint32_t R_tilde = 0;
  uint64_t sweeps = 0;
  uint32_t step = 0;
  double beta = 0.0, sum_lnQ = 0.0;
  double last_dbeta = 0.0, last_lnQ = 0.0, last_eps = 0.0;
  uint32_t last_n_culled = 0, last_R_old = 0;
  bool pending_gather = false;
  bool hist_valid = false;
  bool failed = false;
  // pinned staging
  uint32_t* h_hist = nullptr;
  pa::TableEntry* h_table = nullptr;  // staging of the resampling table
  pa::DevScalars* h_sc = nullptr;
  pa::RealScalars* h_rs = nullptr;    // PA_MODEL_GAUSS: after h_sc in the same block
  long long r_Emin_pre = 0;           // PA_MODEL_GAUSS: E_min of the population a queued
                                      // resampling step weighs (its ln Q needs it)
  unsigned long long* h_ovl = nullptr;
  unsigned long long* h_lovl = nullptr;  // 3N + 1 link-overlap counts
  pa_host::MetaU32* h_meta = nullptr;
  unsigned long long* h_gthr = nullptr;  // PA_MODEL_GAUSS16 threshold table staging
  hipEvent_t gthr_copied = nullptr;      // recorded after each copy out of h_gthr
  bool in_batch = false;
  uint32_t flags = 0;                 // PA_FLAG_* of the instance's parameters
  int device = -1;                    // the device current at creation
  hipEvent_t sweep_ev[2] = {nullptr, nullptr};  // PA_FLAG_TIME_SWEEPS: around the last sweep
  bool sweep_timed = false;           // the events bracket a launch not yet read
  double last_sweep_ms = 0.0;
  // pipelined steps (pa_anneal_run): the histogram copy of a queued step, and
  // the family sums of two steps in flight
  hipEvent_t ev_step = nullptr;
  hipEvent_t ev_fam[2] = {nullptr, nullptr};
  unsigned long long* h_eta2 = nullptr;  // pinned, two slots
  int64_t fail_countdown = -1;        // PA_INJECT_FAIL_AFTER: calls left before the failure
};

namespace pa_host {

// Counts one call on a usable instance: with an armed PA_INJECT_FAIL_AFTER
// countdown, the call at which it runs out fails as a HIP error would, before
// anything is queued, and the instance becomes unusable.
inline int count_call(pa_instance* in) {
  if (in->fail_countdown >= 0) {
    if (in->fail_countdown == 0) {
      in->fail_countdown = -1;
      in->failed = true;
      return PA_EDEVICE;
    }
    --in->fail_countdown;
  }
  return PA_OK;
}

}  // namespace pa_host
