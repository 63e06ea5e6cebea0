// pa_tune.cpp -- the sweep autotuner's table: for (coupling model, spin
// layout, L, size class of the launch) the number of waves per tile that
// measured fastest on this device.  Size class = floor(log2(tiles)).  The form of a sweep changes no
// result (every draw is addressed by slot, sweep and site group), only its time.
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>

#include "../../include/pa.h"
#include "pa_internal.hpp"

namespace {

std::mutex g_mu;
std::map<std::tuple<uint32_t, uint32_t, uint32_t, uint32_t>, uint32_t> g_table;

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
  return sweep_split_default(L, tiles);
}

void sweep_split_record(uint32_t model, uint32_t layout, uint32_t L, uint64_t tiles,
                        uint32_t split) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[{model, layout, L, size_class(tiles)}] = split;
}

}  // namespace pa

extern "C" int pa_autotune_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  return PA_OK;
}
