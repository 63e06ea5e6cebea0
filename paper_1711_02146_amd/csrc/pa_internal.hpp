// pa_internal.hpp -- types shared by the HIP kernels and the host side of
// libpa (the C-ABI implementation).  Nothing here is visible to callers.
//
// Method: Amey & Machta, arXiv:1711.02146 (Sec. II annealing loop, Eqs. 1-2
// resampling, Sec. II.A model and observables, Sec. III.A rho_t).
//
// Every kernel works on a set of populations: a device array of DevPop plus a
// Group that maps each workgroup to (member population, block within it).  A
// single instance is a set of one.  Per-launch parameters come either by value
// (calls on one instance) or from a device array indexed by a device step
// counter, so that one captured graph can be replayed for every temperature
// step of a batch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pa {

// Philox stream tags (fourth counter word): one per use of the generator.
constexpr uint32_t kTagInit = 0x494E4954u;  // initial spins
constexpr uint32_t kTagMet = 0x4D455452u;   // Metropolis acceptance draws
constexpr uint32_t kTagRes = 0x52455341u;   // copy-count draws
constexpr uint32_t kTagJ = 0x434F5550u;     // +-J couplings (pa_make_couplings_pm)

constexpr int kWave = 64;          // wavefront width on gfx950; one spin tile = 64 replicas
constexpr int kBlockCounts = 256;  // slots per block in the copy-count / scatter kernels
constexpr int kHistSlots = 4096;   // slots per block of the histogram kernel
constexpr int kWindowLdsLevels = 16384;  // largest E16 window counted in LDS (64 KiB)
constexpr int kMaxL = 16;
// Sweep: per wave, one byte for each of 64 sites x 64 replicas (phase 1 of
// the colour pass: one site per lane): the threshold byte address (+-J) or
// the neighbour pattern (Gaussian couplings).  With the 8 KB tile image at L = 10, eight such areas leave four
// workgroups of eight waves (eight waves per SIMD) in a CU's 160 KB.
constexpr uint32_t kPlaneAreaBytes = 64 * 64;
constexpr uint32_t kLinkCopies = 32;  // partial link-overlap histograms (see launch_link_overlap)
// Energy models.  kModelPm: J = +-1, the energy word of a replica is U, the
// number of unsatisfied bonds (E = 2U - 3N).  kModelGauss16: J = k / 16 with
// k in [-127, 127], the energy word is E16 = -sum_b k_b s_i s_j (E = E16 / 16),
// stored as int32.
constexpr uint32_t kModelPm = 0;
constexpr uint32_t kModelGauss16 = 1;
// kModelReal: real Gaussian couplings (Sec. II.A) carried on the grid 2^-32
// with |J| < 8.  The energy word is the int64 E32 = E 2^32, exact: every sum
// of at most 3N such couplings fits in 49 bits.  Per site (colour-major cm)
// and per pattern y of its six "neighbour differs" bits (bit k: s_i != s_k,
// k in the order +x,-x,+y,-y,+z,-z), he[cm][y] = sum_k k_k (1 - 2 y_k) with
// k_k = J_k 2^32: flipping s_i changes E32 by 2 he, and the site's bond
// energy is -he before and +he after the flip.
constexpr uint32_t kModelReal = 2;
constexpr uint32_t kRealPatterns = 64;  // patterns y per site
// Rows (sites) past the last of the per-(site, pattern) tables: the Gaussian
// colour pass reads one group of four sites past a 64-site chunk ahead, whose
// entries it never uses.
constexpr uint32_t kPatternPadRows = 64;
// Workgroups of the kModelReal weight reductions (grid-stride over the
// replicas), one per CU: measured at L=10, R=5e5, an evaluation of the
// bisection takes 17 us on 256 workgroups, 21 us on 128 and 29 us on 1024
// (each workgroup's arrival costs a device-scope fence and atomic).
constexpr uint32_t kRealSumBlocks = 256;
constexpr int kGaussKMax = 127;
constexpr int kGaussDEMax = 2 * 6 * kGaussKMax;  // largest |dE16| of one flip

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

// LDS address of the tile image in the sweep kernel: right after its 8-entry
// threshold table, which sits at address 0 (the kernel checks both).
constexpr uint32_t kTileLdsBase = 64;

// The same site for phase 1 of the colour passes (lane = site), laid out so
// that nothing needs unpacking: the LDS addresses kTileLdsBase + 8 nb[k] of
// the six neighbours' words, and the coupling bits.  32 bytes: two 16-byte
// loads per lane.
struct PlaneSite {
  uint32_t nb8[6];
  uint32_t jneg;
  uint32_t pad;
};
static_assert(sizeof(PlaneSite) == 32, "PlaneSite must be 32 bytes");

// Device-resident scalars of one population.
struct DevScalars {
  uint32_t R_tilde;       // size of the current population
  uint32_t R_next;        // size after the pending copy step (written by the scan)
  uint32_t err;           // 1: the pending copy step would exceed the capacity;
                          // 2: a kernel found its LDS layout unusable
  uint32_t n_culled;      // replicas with zero copies in the last resampling step
  unsigned long long sum_eta2;  // sum over families of eta^2
  uint32_t check_bad;     // energy check: replicas whose stored word differs from the spins'
  uint32_t dead;          // batch runs: set when a step overflowed; later steps skip it
  int32_t E_lo, E_hi;     // kModelGauss16: lowest / highest E16 of the population
  uint32_t pad[6];
};
static_assert(sizeof(DevScalars) == 64, "DevScalars is 64 bytes");

// Device scalars of a kModelReal population (after DevScalars in the same
// block, so one copy brings both to the host).  The reductions over replicas
// finish in the last workgroup to arrive (counter `done`, reset by it).
struct RealScalars {
  long long E_min;             // lowest energy word (k_rstats)
  unsigned long long sumE_lo;  // sum of the energy words, a 128-bit two's-complement
  long long sumE_hi;           //   integer (low and high word)
  uint32_t n_at_min;           // replicas at E_min
  uint32_t done;               // workgroups arrived at the current reduction
  double S;                    // sum of the weights of dbeta (Eq. 2, fixed point, rounded)
  double eps;                  // culled fraction (Sec. III.C) of the last copy-count pass
  double dbeta;                // the step the bisection evaluates next
  double lo, hi;               // bisection interval
  double rem, target;          // remaining range and culling target of the bisection
  uint32_t phase;              // evaluations the bisection has finished
  int32_t result;              // 0 running, 1 whole range, 2 bisected (lo), -1 impossible
  uint32_t pad[4];
};
static_assert(sizeof(RealScalars) == 112, "RealScalars is 112 bytes");

// One workgroup's share of a kModelReal reduction.
struct RealPartial {
  unsigned long long lo;  // fixed-point sum (unsigned) or energy sum (signed), low word
  unsigned long long hi;  //   high word
  long long m;            // lowest energy word
  uint32_t c;             // replicas at m
  uint32_t pad;
};
static_assert(sizeof(RealPartial) == 32, "RealPartial is 32 bytes");

// One energy level of the resampling table (Sec. II copy rule): a replica
// at that level gets fl copies, and one more iff a 53-bit draw is below T.
// The two live together so that the table goes to the device in one copy.
struct TableEntry {
  unsigned long long T;  // ceil(frac(tau_j) 2^53)
  uint32_t fl;           // floor(tau_j)
  uint32_t pad;
};
static_assert(sizeof(TableEntry) == 16, "TableEntry is 16 bytes");

// The occupied range of a resampling table passed by value to the copy-count
// kernel of a single population, when it fits: no separate upload (and no
// dispatch between the upload and the kernel).  Entry e[j - j0] is level j.
constexpr uint32_t kInlineLevels = 224;
struct InlineTable {
  uint32_t j0, n;
  uint32_t pad[2];
  TableEntry e[kInlineLevels];
};
static_assert(sizeof(InlineTable) == 16 + 16 * kInlineLevels, "InlineTable layout");

// Device pointers of one population (all inside its workspace).
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
  struct TableEntry* table;     // n_levels: the resampling table by energy level
  const SiteEntry* sites;       // N entries, colour-major
  const PlaneSite* psites;      // N entries, colour-major (phase 1 of the colour passes)
  const uint16_t* cm_of_site;   // N entries: lexicographic site -> colour-major index
  const unsigned long long* rowj;  // 2 L^2 row words: bit 6q + k set iff the bond from
                                   // site q of row (colour, y, z) to neighbour k is -1
  unsigned long long* ovl_hist; // 65 bins, scratch of the overlap histogram
  unsigned long long* lovl_hist;  // 3N + 1 bins, scratch of the link-overlap histogram
  uint32_t* lovl_part;            // kLinkCopies x (3N + 1) partial link-overlap counts
  DevScalars* sc;
  uint32_t model;               // kModelPm or kModelGauss16
  uint32_t rowk_stride;         // kModelGauss16: bytes per row of rowk (6 L/2 rounded up to 4)
  const int8_t* rowk;           // kModelGauss16: 2 L^2 rows; byte 6q + k of a row is the
                                // coupling k of its site q to neighbour k (J = k / 16)
  const unsigned long long* gthr;  // kModelGauss16: thr[d] = floor(2^32 exp(-beta d / 16)),
                                   // d = 0..kGaussDEMax, for the coming sweep
  const uint16_t* gaddr;            // kModelGauss16: 16 max(he16[cm][y], 0), N x 64, with he16
                                   // the he of kModelReal in units 1/16: the byte offset of the
                                   // move's threshold in the dE16 table (dE16 = 2 he16)
  const long long* rhe;            // kModelReal: he[cm][y], N x 64 (see kModelReal)
  unsigned long long* rthr;        // kModelReal: Metropolis threshold of (cm, y) for the
                                   // coming sweep, N x 64
  uint32_t* rthr32;                // kModelReal: min(thr, 2^32 - 1) of the same (cm, y): the
                                   // sweep's table (see pattern_thr)
  RealScalars* rs;                 // kModelReal: scalars of the weight reductions
  RealPartial* rpart;              // kModelReal: one per workgroup of kBlockCounts slots
};

// Parameters of one population for one launch.
struct PopStep {
  unsigned long long thr[3];  // Metropolis thresholds (dE = 4, 8, 12): accept iff word < thr
  const double* erow;         // device table path: erow[d] = exp(-dbeta * 2d), d = 0..3N
  uint32_t t0;                // population sweep counter at the first sweep
  uint32_t n_sweeps;
  uint32_t gather;            // 1: the sweep applies the pending copy step (size R_next)
  uint32_t cur;               // buffer holding the population at the start of the launch
  uint32_t step;              // resampling step index k (copy-count Philox counter)
  uint32_t flags;             // kStepSticky: an overflow marks the population dead; kStepHist
  double dbeta;               // kModelReal: the resampling step of the copy-count pass
};
static_assert(sizeof(PopStep) == 64, "PopStep is 64 bytes");
constexpr uint32_t kStepSticky = 1u;
// kStepHist (+-J): the scan also clears the energy histogram and the family
// sum, for the histogram and family kernels that follow the sweep (no
// separate clearing launch).
constexpr uint32_t kStepHist = 2u;

// What a batch records for one population at one temperature step.
struct StepRecord {
  double S;                // sum_j h_j w_j of the resampling table (Eq. 2, shifted)
  double eps;              // culling fraction of the step (Sec. III.C)
  long long sumE;          // sum over the post-sweep population of E (integer)
  unsigned long long sum_eta2;
  int32_t jmin;            // lowest occupied level before resampling
  uint32_t R_old;          // population size before resampling
  uint32_t R_new;          // population size after resampling and sweeps
  uint32_t n_culled;
  int32_t E_min;           // lowest energy after the sweeps
  uint32_t status;         // 0 ok, 1 capacity overflow (population dead from here on),
                           // 2 the sweep kernel found its LDS layout unusable (dead)
  uint32_t n_at_E_min;     // replicas at E_min
  uint32_t pad;
};
static_assert(sizeof(StepRecord) == 64, "StepRecord is 64 bytes");

// A set of populations as the kernels see it.
struct BatchDev {
  const DevPop* pops;         // n_pops descriptors
  const PopStep* steps;       // per-step parameters [n][n_pops], or nullptr: use `single`
  const uint32_t* step_ctr;   // index of the current step into `steps`
  StepRecord* records;        // [n][n_pops] results of batch steps, or nullptr
  unsigned long long* qhist;  // [n][n_pairs][65] overlap histograms, or nullptr
  uint32_t n_pops;
  uint32_t n_pairs;
  PopStep single;             // parameters of a call on one population
};

// Workgroup -> population map of one launch: member m owns workgroups
// start[m] .. start[m+1]-1 and is population pop[m] of the set.
struct Group {
  const uint32_t* pop;
  const uint32_t* start;  // n + 1 entries, start[0] = 0
  uint32_t n;
  uint32_t blocks;        // start[n]
};

// Launchers (pa_kernels.hip).  All are asynchronous on `stream`.
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t stream);

// Diagnostics (pa_probe_ceilings): kProbeThreads lanes, each writing one word
// of `out`; the VALU probe issues kProbeValuOpsPerIter instructions per
// iteration (form 0: v_add_u32, form 1: v_bfe_u32), the Philox probe makes
// `calls` Metropolis Philox calls (4 draws each).
constexpr uint32_t kProbeThreads = 2048 * 256;
constexpr int kProbeValuOpsPerIter = 32;
hipError_t launch_probe_valu(uint32_t* out, uint32_t iters, uint32_t form, hipStream_t stream);
hipError_t launch_probe_philox(uint32_t* out, uint32_t calls, hipStream_t stream);
hipError_t launch_init(const DevPop& P, uint32_t cur, hipStream_t stream);
hipError_t launch_zero_acc(const BatchDev& B, const Group& per_pop, hipStream_t stream);
hipError_t launch_hist(const BatchDev& B, const Group& g, uint32_t max_levels, bool post,
                       hipStream_t stream);
hipError_t launch_table(const BatchDev& B, const Group& per_pop, hipStream_t stream);
hipError_t launch_counts(const BatchDev& B, const Group& g, hipStream_t stream);
// the same with the table's occupied range passed by value (single populations)
hipError_t launch_counts_inline(const BatchDev& B, const Group& g, const InlineTable& t,
                                hipStream_t stream);
hipError_t launch_scan(const BatchDev& B, const Group& per_pop, hipStream_t stream);
hipError_t launch_scatter(const BatchDev& B, const Group& g, hipStream_t stream);
// k_scan and k_scatter of one population in one launch (g: its slot blocks)
hipError_t launch_scan_scatter(const BatchDev& B, const Group& g, hipStream_t stream);
// sweep launch over the populations of one (layout, L, model) group: one tile
// per workgroup of `split` (4 or 8) waves; g's blocks are blocks_sweep(capacity)
hipError_t launch_sweep(const BatchDev& B, const Group& g, uint32_t layout, uint32_t L,
                        uint32_t split, uint32_t model, hipStream_t stream);
hipError_t launch_family(const BatchDev& B, const Group& g, bool post, hipStream_t stream);
hipError_t launch_record(const BatchDev& B, const Group& per_pop, hipStream_t stream);
// cur_a / cur_b: the two populations' buffers when B carries no per-step parameters
hipError_t launch_overlap(const BatchDev& B, const Group& pairs, const uint32_t* pair_pops,
                          uint32_t layout, bool post, uint32_t cur_a, uint32_t cur_b,
                          hipStream_t stream);
// energy word of every replica of buffer cur recomputed from its spins: stored
// (check == false), or compared with the stored word, the number of replicas
// that differ added to sc->check_bad (check == true)
hipError_t launch_energy(const BatchDev& B, const Group& g, uint32_t layout, uint32_t L,
                         uint32_t model, bool check, hipStream_t stream);
// link-overlap histogram of slot i of a against slot i of b, i < min of their
// R~ (read on the device): the pairs count into kLinkCopies partial histograms
// part[kLinkCopies][3N + 1] (u32, cleared by the host first), which are then
// summed into hist[D], D = 0..3N
hipError_t launch_link_overlap(const DevPop& a, const DevPop& b, uint32_t cur_a, uint32_t cur_b,
                               uint32_t* part, unsigned long long* hist, hipStream_t stream);
// kModelGauss16: E_lo / E_hi of every member (zero_acc resets them first) and the
// histogram h[E16 - E_lo] (global atomics; the host clears the window first),
// both over the current buffer of a call on single instances
// kModelGauss16 (groups of kHistSlots slots per workgroup): the population's
// E16 range into E_lo / E_hi, then the histogram over the n_win-level window.
hipError_t launch_minmax(const BatchDev& B, const Group& g, hipStream_t stream);
hipError_t launch_hist_window(const BatchDev& B, const Group& g, uint32_t n_win,
                              hipStream_t stream);
hipError_t launch_advance(uint32_t* step_ctr, hipStream_t stream);

// kModelReal (pa_real.hip), single populations, on the current buffer:
// thresholds of every (site, pattern) at beta for the coming sweep
hipError_t launch_real_thresholds(const DevPop& P, double beta, hipStream_t stream);
// E_min, replicas at E_min and the sum of the energy words into P.rs
hipError_t launch_real_stats(const BatchDev& B, const Group& slots, hipStream_t stream);
// the sum S of the weights exp(-dbeta (E - E_min)) at the step's dbeta into P.rs->S
hipError_t launch_real_sum(const BatchDev& B, const Group& slots, hipStream_t stream);
// the constant-culling bisection (Sec. III.C): set up for the remaining range
// and target, then one evaluation (culled mass at the current candidate, the
// weight sums of the two that can follow, the decision) per
// launch_real_bisect_eval; 66 of them finish it (P.rs->result).  Each
// evaluation runs on `blocks` workgroups (at most kRealSumBlocks: the
// partials hold three sums each) over one population, whose buffers it takes
// as arguments, so that its first loads need no descriptor read before them.
struct RevalArgs {
  const long long* E;     // energy words of the population's current buffer
  const DevScalars* sc;   // R_tilde
  RealScalars* rs;        // the search state
  RealPartial* rpart;     // 3 x blocks partials
  uint32_t R;             // target population size
  uint32_t capacity;      // slots per buffer (every slot below it is allocated)
};
hipError_t launch_real_bisect_init(const DevPop& P, double rem, double target,
                                   hipStream_t stream);
hipError_t launch_real_bisect_eval(const RevalArgs& a, uint32_t blocks, hipStream_t stream);
// copy counts of the step (after launch_real_sum at its dbeta): counts, block
// sums and culled counts as k_counts, and the culled fraction into P.rs->eps
// (`slots`: at most kRealSumBlocks workgroups, each over every nb-th slot block)
hipError_t launch_real_counts(const BatchDev& B, const Group& slots, hipStream_t stream);

// Blocks each population needs in each kind of launch.
inline uint32_t blocks_hist(uint32_t capacity) { return (capacity + kHistSlots - 1) / kHistSlots; }
inline uint32_t blocks_slots(uint32_t capacity) { return capacity / kBlockCounts; }
// One block per tile, rounded up to a multiple of 8 so that every population
// of a launch starts at a block number divisible by the XCD count (the extra
// blocks find no replicas and leave).
inline uint32_t blocks_sweep(uint32_t capacity) { return (capacity / 64 + 7) / 8 * 8; }
// Waves per tile of a sweep launch over `tiles` tiles of linear size L, from
// timings on MI355X (both layouts, beta = 1, 10 sweeps; the same two-phase
// colour pass for every coupling model): eight waves from L = 10 up, and on
// smaller lattices while the launch is too small to fill the chip with four
// (fewer than 256 (L - 2) tiles: 512 at L = 4, 1024 at L = 6, 1536 at L = 8);
// four otherwise, where more resident tiles per CU pay (L = 4, 4096 tiles:
// 0.13 against 0.19 ms).
inline uint32_t sweep_split_default(uint32_t model, uint32_t L, uint64_t tiles) {
  (void)model;
  return (L >= 10 || tiles < 256ull * (L - 2)) ? 8u : 4u;
}
// The split a launch uses: the autotuner's choice for (model, layout, L, size
// class of `tiles`) when one was measured in this process, else the default (pa_tune.cpp).
uint32_t sweep_split_for(uint32_t model, uint32_t layout, uint32_t L, uint64_t tiles);
void sweep_split_record(uint32_t model, uint32_t layout, uint32_t L, uint64_t tiles,
                        uint32_t split);

// Spin layout of a population created with the library's choice, when the
// autotuner has not timed its shape: bit-packed (one bit per spin, 64
// replicas per word) for every shape; values are PA_LAYOUT_INT8 = 1 and
// PA_LAYOUT_BITPACK64 = 2.
inline uint32_t layout_default(uint32_t, uint32_t, uint64_t) { return 2u; }
// The autotuner's layout for (model, L, size class of `tiles`) when one was
// measured or pinned in this process, else layout_default (pa_tune.cpp).
uint32_t layout_for(uint32_t model, uint32_t L, uint64_t tiles);
void layout_record(uint32_t model, uint32_t L, uint64_t tiles, uint32_t layout);

}  // namespace pa
