// pa_tune.cpp -- device measurement: the autotuner's two tables and the probes
// of the device's VALU and Philox ceilings.  The split table holds, per
// coupling model, spin layout, L and size class of a sweep launch, the number
// of waves per tile that measured fastest on this device; the layout table
// holds, per coupling model, L and size class, the spin layout whose sweep
// measured fastest (the layout PA_LAYOUT_AUTO resolves to at creation).  Size
// class = floor(log2(tiles)).  Neither choice changes a result (every draw is
// addressed by slot, sweep and site group, and both layouts hold the same
// spins), only the time.
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>

#include "../../include/pa.h"
#include "pa_internal.hpp"

namespace {

std::mutex g_mu;
std::map<std::tuple<uint32_t, uint32_t, uint32_t, uint32_t>, uint32_t> g_table;
std::map<std::tuple<uint32_t, uint32_t, uint32_t>, uint32_t> g_layouts;

uint32_t size_class(uint64_t tiles) {
  uint32_t c = 0;
  while (tiles > 1) {
    tiles >>= 1;
    ++c;
  }
  return c;
}

}  // namespace

namespace pa {

uint32_t sweep_split_for(uint32_t model, uint32_t layout, uint32_t L, uint64_t tiles) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const auto it = g_table.find({model, layout, L, size_class(tiles)});
    if (it != g_table.end()) return it->second;
  }
  return sweep_split_default(model, L, tiles);
}

void sweep_split_record(uint32_t model, uint32_t layout, uint32_t L, uint64_t tiles,
                        uint32_t split) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[{model, layout, L, size_class(tiles)}] = split;
}

uint32_t layout_for(uint32_t model, uint32_t L, uint64_t tiles) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const auto it = g_layouts.find({model, L, size_class(tiles)});
    if (it != g_layouts.end()) return it->second;
  }
  return layout_default(model, L, tiles);
}

void layout_record(uint32_t model, uint32_t L, uint64_t tiles, uint32_t layout) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_layouts[{model, L, size_class(tiles)}] = layout;
}

}  // namespace pa

extern "C" int pa_layout_choice(uint32_t model, uint32_t L, uint32_t R, uint32_t* layout_out) {
  if (!layout_out) return PA_EINVAL;
  if (model != PA_MODEL_PM && model != PA_MODEL_GAUSS16 && model != PA_MODEL_GAUSS) return PA_EINVAL;
  if (L < 4 || L > (uint32_t)pa::kMaxL || (L & 1u) || R == 0) return PA_EINVAL;
  *layout_out = pa::layout_for(model, L, ((uint64_t)R + 63) / 64);
  return PA_OK;
}

extern "C" int pa_autotune_set_layout(uint32_t model, uint32_t L, uint64_t tiles, uint32_t layout) {
  if (model != PA_MODEL_PM && model != PA_MODEL_GAUSS16 && model != PA_MODEL_GAUSS) return PA_EINVAL;
  if (layout != PA_LAYOUT_INT8 && layout != PA_LAYOUT_BITPACK64) return PA_EINVAL;
  if (L < 4 || L > (uint32_t)pa::kMaxL || (L & 1u) || tiles == 0) return PA_EINVAL;
  pa::layout_record(model, L, tiles, layout);
  return PA_OK;
}

extern "C" int pa_autotune_set(uint32_t model, uint32_t layout, uint32_t L, uint64_t tiles,
                               uint32_t split) {
  if (model != PA_MODEL_PM && model != PA_MODEL_GAUSS16 && model != PA_MODEL_GAUSS) return PA_EINVAL;
  if (layout != PA_LAYOUT_INT8 && layout != PA_LAYOUT_BITPACK64) return PA_EINVAL;
  if (L < 4 || L > (uint32_t)pa::kMaxL || (L & 1u) || tiles == 0) return PA_EINVAL;
  if (split != 4 && split != 8) return PA_EINVAL;
  pa::sweep_split_record(model, layout, L, tiles, split);
  return PA_OK;
}

extern "C" int pa_autotune_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  g_layouts.clear();
  return PA_OK;
}

extern "C" size_t pa_probe_scratch_bytes(void) { return (size_t)pa::kProbeThreads * 4; }

extern "C" int pa_probe_ceilings(void* d_scratch, size_t bytes, void* hip_stream,
                                 pa_ceilings* out) {
  if (!d_scratch || !out || bytes < pa_probe_scratch_bytes()) return PA_EINVAL;
  if (reinterpret_cast<uintptr_t>(d_scratch) % 4) return PA_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  uint32_t* o = static_cast<uint32_t*>(d_scratch);
  constexpr uint32_t kIters = 4096, kCalls = 2048, kWarm = 2, kTimed = 5;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return PA_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return PA_EDEVICE;
  }
  // average launch time of `launch` in ms, or a negative value on a HIP error
  auto time_of = [&](auto launch) -> float {
    for (uint32_t w = 0; w < kWarm; ++w)
      if (launch() != hipSuccess) return -1.0f;
    float sum = 0.0f;
    for (uint32_t r = 0; r < kTimed; ++r) {
      float ms = 0.0f;
      if (hipEventRecord(e0, s) != hipSuccess || launch() != hipSuccess ||
          hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        return -1.0f;
      sum += ms;
    }
    return sum / (float)kTimed;
  };
  const float ms_valu = time_of([&] { return pa::launch_probe_valu(o, kIters, 0u, s); });
  const float ms_valu3 =
      ms_valu > 0.0f ? time_of([&] { return pa::launch_probe_valu(o, kIters, 1u, s); }) : -1.0f;
  const float ms_philox =
      ms_valu3 > 0.0f ? time_of([&] { return pa::launch_probe_philox(o, kCalls, s); }) : -1.0f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!(ms_valu > 0.0f) || !(ms_valu3 > 0.0f) || !(ms_philox > 0.0f)) return PA_EDEVICE;
  const double lane_instr = (double)pa::kProbeThreads * kIters * pa::kProbeValuOpsPerIter;
  out->valu_lane_ops_per_s = lane_instr / (ms_valu * 1e-3);
  out->valu3_lane_ops_per_s = lane_instr / (ms_valu3 * 1e-3);
  out->philox_draws_per_s = (double)pa::kProbeThreads * kCalls * 4.0 / (ms_philox * 1e-3);
  return PA_OK;
}
