// pa_internal.hpp -- types shared by the HIP kernels and the host side of
// libpa (the C-ABI implementation).  Nothing here is visible to callers.
//
// Method: Amey & Machta, arXiv:1711.02146 (Sec. II annealing loop, Eqs. 1-2
// resampling, Sec. II.A model and observables, Sec. III.A rho_t).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pa {

// Philox stream tags (fourth counter word): one per use of the generator.
constexpr uint32_t kTagInit = 0x494E4954u;  // initial spins
constexpr uint32_t kTagMet = 0x4D455452u;   // Metropolis acceptance draws
constexpr uint32_t kTagRes = 0x52455341u;   // copy-count draws

constexpr int kWave = 64;          // wavefront width on gfx950; one spin tile = 64 replicas
constexpr int kBlockCounts = 256;  // slots per block in the copy-count / scatter kernels
constexpr int kMaxL = 16;

// One lattice site in colour-major order (cm): colour-0 sites first, then
// colour-1 sites, each in lexicographic order; for even L, cm = c*N/2 + (site >> 1).
// nb[k] are the colour-major indices of the six neighbours (+x,-x,+y,-y,+z,-z),
// bit k of jneg is set when the coupling to neighbour k is -1, site is the
// lexicographic index.  16 bytes: one scalar load per site.
struct SiteEntry {
  uint16_t nb[6];
  uint16_t jneg;
  uint16_t site;
};
static_assert(sizeof(SiteEntry) == 16, "SiteEntry must be 16 bytes");

// Device-resident scalars of one population.
struct DevScalars {
  uint32_t R_tilde;       // size of the current population
  uint32_t R_next;        // size after the pending copy step (written by the scan)
  uint32_t err;           // 1: the pending copy step would exceed the capacity
  uint32_t n_culled;      // replicas with zero copies in the last resampling step
  unsigned long long sum_eta2;  // sum over families of eta^2
  uint32_t n_families;    // families with eta > 0
  uint32_t pad[9];
};
static_assert(sizeof(DevScalars) == 64, "DevScalars is 64 bytes");

// Device pointers of one population (all inside the caller's workspace).
struct DevPop {
  uint32_t L, N, R, capacity;   // capacity: slots per buffer, a multiple of kBlockCounts
  uint32_t layout;              // PA_LAYOUT_INT8 or PA_LAYOUT_BITPACK64
  uint32_t n_levels;            // 3N + 1
  uint32_t n_blocks;            // capacity / kBlockCounts
  uint32_t cap_limit;           // a resampled population may not exceed this (<= capacity)
  uint64_t seed;
  void* spins[2];               // tile-major spin buffers (see pa.h)
  uint32_t* U[2];
  uint32_t* fam[2];
  uint32_t* counts;             // n_i of the last resampling step
  uint32_t* offsets;            // exclusive scan of counts
  uint32_t* src;                // new slot -> old slot of the pending copy step
  uint32_t* block_sums;         // per block of kBlockCounts slots
  uint32_t* block_offsets;
  uint32_t* block_culled;
  uint32_t* hist;               // n_levels
  uint32_t* table_fl;           // n_levels: floor(tau_j)
  unsigned long long* table_T;  // n_levels: ceil(frac(tau_j) 2^53)
  const SiteEntry* sites;       // N entries, colour-major
  const uint16_t* cm_of_site;   // N entries: lexicographic site -> colour-major index
  const unsigned long long* rowj;  // 2 L^2 row words: bit 6q + k set iff the bond from
                                   // site q of row (colour, y, z) to neighbour k is -1
  unsigned long long* ovl_hist; // 65 bins, scratch of the overlap histogram
  DevScalars* sc;
};

// Per-launch sweep parameters.
struct SweepParams {
  uint64_t thr[3];      // thresholds for dE = 4, 8, 12: accept iff word < thr
  uint32_t t0;          // population sweep counter at the first sweep
  uint32_t n_sweeps;
  uint32_t gather;      // 1: new slot j takes old slot src[j]; population size R_next
  uint32_t cur;         // buffer holding the current population
};

// Launchers (pa_kernels.hip).  All are asynchronous on `stream`.
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t stream);
hipError_t launch_init(const DevPop& P, uint32_t cur, hipStream_t stream);
hipError_t launch_hist(const DevPop& P, uint32_t cur, hipStream_t stream);
hipError_t launch_counts(const DevPop& P, uint32_t cur, uint32_t step, hipStream_t stream);
hipError_t launch_scan(const DevPop& P, hipStream_t stream);
hipError_t launch_scatter(const DevPop& P, hipStream_t stream);
hipError_t launch_sweep(const DevPop& P, const SweepParams& sp, hipStream_t stream);
hipError_t launch_family(const DevPop& P, uint32_t cur, hipStream_t stream);
hipError_t launch_overlap(const DevPop& A, uint32_t cur_a, const DevPop& B, uint32_t cur_b,
                          unsigned long long* hist65, hipStream_t stream);
hipError_t launch_energy(const DevPop& P, uint32_t cur, hipStream_t stream);

}  // namespace pa
