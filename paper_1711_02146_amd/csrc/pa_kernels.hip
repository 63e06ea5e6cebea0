// pa_kernels.hip -- gfx950 kernels of the population-annealing hot path.
//
// Method: Amey & Machta, arXiv:1711.02146.
//   Sec. II    annealing loop: resample (Eqs. 1-2, nearest-integer copy
//              counts, copies inherit family labels), then MCMC sweeps.
//   Sec. II.A  3D +-J Edwards-Anderson model on the periodic cubic lattice.
//   Sec. III.A family statistic rho_t.
//
// Execution model.  A spin tile is 64 replicas = one wavefront: lane l owns
// replica (tile*64 + l).  Inside the sweep kernel the tile lives in LDS as one
// 64-bit word per site (colour-major order), bit l = spin of lane l
// (1 <=> s = -1).  Each lane reads the 32-bit half holding its bit, so the
// local field, the acceptance test and the Philox draw are per lane, and the
// flips of the 64 replicas at a site come back as one wave ballot, XORed into
// the site word.  Every draw is a Philox4x32-10 word addressed by (slot,
// sweep, site group, tag), so the result is independent of the launch shape.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pa_internal.hpp"

namespace pa {
namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies (round multipliers 0xD2511F53, 0xCD9E8D57), a swap of
// the halves and an XOR with the other counter words and the round key; the
// key advances by the Weyl constants 0x9E3779B9, 0xBB67AE85 between rounds.
// ---------------------------------------------------------------------------
struct Words4 {
  uint32_t w[4];
};

// a ^ b ^ c in one VALU instruction (gfx950 v_bitop3_b32, truth table 0x96);
// c must be wave-uniform (it is read from an SGPR).
__device__ __forceinline__ uint32_t xor3_s(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

__device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t pa = (uint64_t)0xD2511F53u * c0;  // one v_mad_u64_u32
    const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = xor3_s((uint32_t)(pb >> 32), c1, k0);
    const uint32_t n2 = xor3_s((uint32_t)(pa >> 32), c3, k1);
    c0 = n0;
    c1 = (uint32_t)pb;
    c2 = n2;
    c3 = (uint32_t)pa;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Words4 o;
  o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
  return o;
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint32_t bit_of(uint32_t word, uint32_t pos) {
  return (word >> pos) & 1u;
}

// A SiteEntry read as one 16-byte word (a single scalar load when uniform).
struct SiteWords {
  uint32_t nb[6];
  uint32_t jneg;
};

__device__ __forceinline__ SiteWords load_site(const SiteEntry* __restrict__ sites, uint32_t cm) {
  const uint4 w = reinterpret_cast<const uint4*>(sites)[cm];
  SiteWords e;
  e.nb[0] = w.x & 0xFFFFu; e.nb[1] = w.x >> 16;
  e.nb[2] = w.y & 0xFFFFu; e.nb[3] = w.y >> 16;
  e.nb[4] = w.z & 0xFFFFu; e.nb[5] = w.z >> 16;
  e.jneg = w.w & 0xFFFFu;
  return e;
}

// --- spin tile <-> LDS -----------------------------------------------------
// LDS image of a tile: lds[2*cm + h] is the h-th 32-bit half of the 64-bit
// word of site cm (h = lane >> 5 holds lane's bit at position lane & 31).

// New slot j (this lane) takes the spins of old slot src (a gather; src = j
// for a plain copy).  Lanes with valid == false contribute zero bits.
template <int LAYOUT>
__device__ void load_tile_gather(uint32_t* lds, const void* spins_old, uint32_t N, uint32_t src,
                                 bool valid) {
  const uint32_t lane = lane_id();
  const uint32_t stile = src >> 6;
  if (LAYOUT == 2) {  // PA_LAYOUT_BITPACK64
    const uint32_t* w32 = static_cast<const uint32_t*>(spins_old);
    const size_t base = (size_t)stile * N * 2 + ((src >> 5) & 1u);
    const uint32_t pos = src & 31u;
    for (uint32_t cm = 0; cm < N; ++cm) {
      const uint32_t b = valid ? bit_of(w32[base + 2 * (size_t)cm], pos) : 0u;
      const unsigned long long m = __ballot(b);
      if (lane == 0) {
        lds[2 * cm] = (uint32_t)m;
        lds[2 * cm + 1] = (uint32_t)(m >> 32);
      }
    }
  } else {  // PA_LAYOUT_INT8
    const int8_t* s8 = static_cast<const int8_t*>(spins_old);
    const size_t base = (size_t)stile * N * 64 + (src & 63u);
    for (uint32_t cm = 0; cm < N; ++cm) {
      const uint32_t b = valid ? (s8[base + 64 * (size_t)cm] < 0 ? 1u : 0u) : 0u;
      const unsigned long long m = __ballot(b);
      if (lane == 0) {
        lds[2 * cm] = (uint32_t)m;
        lds[2 * cm + 1] = (uint32_t)(m >> 32);
      }
    }
  }
  __syncthreads();
}

template <int LAYOUT>
__device__ void store_tile(const uint32_t* lds, void* spins_new, uint32_t N, uint32_t tile) {
  const uint32_t lane = lane_id();
  if (LAYOUT == 2) {
    uint2* w = static_cast<uint2*>(spins_new) + (size_t)tile * N;
    for (uint32_t cm = lane; cm < N; cm += kWave) w[cm] = make_uint2(lds[2 * cm], lds[2 * cm + 1]);
  } else {
    int8_t* s8 = static_cast<int8_t*>(spins_new) + (size_t)tile * N * 64 + lane;
    const uint32_t h = lane >> 5, pos = lane & 31u;
    for (uint32_t cm = 0; cm < N; ++cm)
      s8[64 * (size_t)cm] = bit_of(lds[2 * cm + h], pos) ? (int8_t)-1 : (int8_t)1;
  }
}

// Number of unsatisfied bonds of this lane's replica: every bond once, as the
// +x, +y, +z bond of its lower site.  A bond is unsatisfied iff
// J s_i s_j = -1, i.e. the XOR of the two spin bits and the coupling bit is 1.
__device__ uint32_t tile_energy(const uint32_t* lds, const SiteEntry* __restrict__ sites,
                                uint32_t N) {
  const uint32_t lane = lane_id();
  const uint32_t h = lane >> 5, pos = lane & 31u;
  uint32_t U = 0;
  for (uint32_t cm = 0; cm < N; ++cm) {
    const SiteWords e = load_site(sites, cm);
    const uint32_t b = bit_of(lds[2 * cm + h], pos);
#pragma unroll
    for (int k = 0; k < 6; k += 2) {
      const uint32_t bn = bit_of(lds[2 * e.nb[k] + h], pos);
      U += b ^ bn ^ ((e.jneg >> k) & 1u);
    }
  }
  return U;
}

// One colour pass of the checkerboard Metropolis update on the LDS tile,
// walked row by row.  For even L, the sites of colour c in row (y, z) are
// x = 2q + p, q = 0..L/2-1, p = (c + y + z) & 1, with colour-major indices
// c*N/2 + (L/2)(y + L z) + q.  Their neighbours of the other colour are, in
// that colour's rank order: +x at q' = (q + p) mod L/2 and -x at
// (q + p - 1) mod L/2 of the same row, and rank q of the rows (y+-1, z) and
// (y, z+-1).  With L a compile-time constant every neighbour is an immediate
// offset from six per-row base addresses.
//
// nu = number of unsatisfied bonds at the site (bond unsatisfied iff own bit
// ^ neighbour bit ^ [J = -1]); flipping changes the energy by dE = 12 - 4 nu,
// so the move is accepted iff its draw is below thr_of_nu[nu]:
// floor(2^32 exp(-beta dE)) for nu = 0, 1, 2 and 2^32 (always) for nu >= 3.
// Consecutive colour-major indices 4g .. 4g+3 share one Philox call; word
// cm & 3 belongs to site cm.  A group can straddle two rows, so the four words
// are carried from row to row.
struct RowCtx {
  uint32_t* lds;
  const unsigned long long* thr_of_nu;
  uint32_t h, pos;       // this lane's half of a site word and its bit
  uint32_t slot, t, k0, k1;
  bool any_draw;
  Words4 d;              // Philox words of the current site group
};

template <int L, int P, int PH>
__device__ __forceinline__ void row_pass(RowCtx& c, uint32_t cm_row, uint32_t oth_x,
                                         uint32_t oth_py, uint32_t oth_my, uint32_t oth_pz,
                                         uint32_t oth_mz, unsigned long long jrow) {
  constexpr int H = L / 2;
  uint32_t* const a_own = c.lds + 2 * cm_row + c.h;
  const uint32_t* const a_x = c.lds + 2 * oth_x + c.h;
  const uint32_t* const a_py = c.lds + 2 * oth_py + c.h;
  const uint32_t* const a_my = c.lds + 2 * oth_my + c.h;
  const uint32_t* const a_pz = c.lds + 2 * oth_pz + c.h;
  const uint32_t* const a_mz = c.lds + 2 * oth_mz + c.h;
  const uint32_t jlo = (uint32_t)jrow, jhi = (uint32_t)(jrow >> 32);
#pragma unroll
  for (int q = 0; q < H; ++q) {
    if (((PH + q) & 3) == 0 && c.any_draw)
      c.d = philox10(c.slot, c.t, (cm_row + q) >> 2, kTagMet, c.k0, c.k1);
    const uint32_t own = a_own[2 * q];
    const uint32_t nb[6] = {a_x[2 * ((q + P) % H)], a_x[2 * ((q + P + H - 1) % H)],
                            a_py[2 * q], a_my[2 * q], a_pz[2 * q], a_mz[2 * q]};
    uint32_t n = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int bit = 6 * q + k;  // coupling bit of (site q, neighbour k) in the row word
      const uint32_t jm = bit < 32 ? (uint32_t)((int32_t)(jlo << (31 - bit)) >> 31)
                                   : (uint32_t)((int32_t)(jhi << (63 - bit)) >> 31);
      n += __builtin_amdgcn_ubfe(xor3_s(nb[k], own, jm), c.pos, 1);
    }
    asm("" : "+v"(n));  // keep the table index a single value
    const bool acc = (unsigned long long)c.d.w[(PH + q) & 3] < c.thr_of_nu[n];
    const unsigned long long f = __ballot(acc);
    const uint32_t fh = c.h ? (uint32_t)(f >> 32) : (uint32_t)f;
    if (c.pos == 0) a_own[2 * q] = own ^ fh;
  }
}

template <int L>
__device__ void sweep_colour_rows(RowCtx& c, const unsigned long long* __restrict__ rowj,
                                  uint32_t colour) {
  constexpr uint32_t H = L / 2, N = L * L * L;
  const uint32_t own0 = colour * (N / 2), oth0 = (colour ^ 1u) * (N / 2);
  for (uint32_t z = 0; z < (uint32_t)L; ++z) {
    const uint32_t zp = z + 1 == (uint32_t)L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
    for (uint32_t y = 0; y < (uint32_t)L; ++y) {
      const uint32_t yp = y + 1 == (uint32_t)L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
      const uint32_t r0 = H * (y + L * z);
      const uint32_t cm_row = __builtin_amdgcn_readfirstlane(own0 + r0);
      const uint32_t ox = oth0 + r0;
      const uint32_t opy = oth0 + H * (yp + L * z), omy = oth0 + H * (ym + L * z);
      const uint32_t opz = oth0 + H * (y + L * zp), omz = oth0 + H * (y + L * zm);
      const unsigned long long jrow = rowj[__builtin_amdgcn_readfirstlane(colour * L * L + y + L * z)];
      const uint32_t p = (colour + y + z) & 1u;
      const uint32_t ph = r0 & 3u;
      // dispatch on the row parity and on where the row starts inside a group
      if constexpr (H % 4 == 0) {
        if (p) row_pass<L, 1, 0>(c, cm_row, ox, opy, omy, opz, omz, jrow);
        else row_pass<L, 0, 0>(c, cm_row, ox, opy, omy, opz, omz, jrow);
      } else if constexpr (H % 2 == 0) {
        switch (p * 4 + ph) {
          case 0: row_pass<L, 0, 0>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
          case 2: row_pass<L, 0, 2>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
          case 4: row_pass<L, 1, 0>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
          default: row_pass<L, 1, 2>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
        }
      } else {
        switch (p * 4 + ph) {
          case 0: row_pass<L, 0, 0>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
          case 1: row_pass<L, 0, 1>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
          case 2: row_pass<L, 0, 2>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
          case 3: row_pass<L, 0, 3>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
          case 4: row_pass<L, 1, 0>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
          case 5: row_pass<L, 1, 1>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
          case 6: row_pass<L, 1, 2>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
          default: row_pass<L, 1, 3>(c, cm_row, ox, opy, omy, opz, omz, jrow); break;
        }
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Initial population at beta = 0 (Sec. II): spin of replica r at site =
// bit 31 of word (site & 3) of Philox(seed; r, site >> 2, 0, INIT).
template <int LAYOUT>
__global__ __launch_bounds__(64) void k_init(DevPop P, uint32_t cur,
                                             const uint16_t* __restrict__ cm_of_site) {
  extern __shared__ uint32_t lds[];
  const uint32_t tile = blockIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t r = tile * 64 + lane;
  const bool valid = r < P.R;
  if (tile * 64 >= P.R) return;
  const uint32_t k0 = (uint32_t)P.seed, k1 = (uint32_t)(P.seed >> 32);
  for (uint32_t g = 0; g < (P.N >> 2); ++g) {
    const Words4 w = philox10(r, g, 0u, kTagInit, k0, k1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const unsigned long long m = __ballot(valid && (w.w[q] >> 31));
      const uint32_t cm = cm_of_site[4 * g + q];
      if (lane == 0) {
        lds[2 * cm] = (uint32_t)m;
        lds[2 * cm + 1] = (uint32_t)(m >> 32);
      }
    }
  }
  __syncthreads();
  const uint32_t U = tile_energy(lds, P.sites, P.N);
  store_tile<LAYOUT>(lds, P.spins[cur], P.N, tile);
  if (valid) {
    P.U[cur][r] = U;
    P.fam[cur][r] = r;
  }
}

// U recomputed from the stored spins (after an import of a state).
template <int LAYOUT>
__global__ __launch_bounds__(64) void k_energy(DevPop P, uint32_t cur) {
  extern __shared__ uint32_t lds[];
  const uint32_t tile = blockIdx.x;
  const uint32_t R = P.sc->R_tilde;
  if (tile * 64 >= R) return;
  const uint32_t j = tile * 64 + lane_id();
  const bool valid = j < R;
  load_tile_gather<LAYOUT>(lds, P.spins[cur], P.N, valid ? j : 0u, valid);
  const uint32_t U = tile_energy(lds, P.sites, P.N);
  if (valid) P.U[cur][j] = U;
}

// Energy histogram h_j = #{i < R~ : U_i = j} (the sum of Eq. 2 regrouped by
// integer level), privatised in LDS.
__global__ __launch_bounds__(256) void k_hist(DevPop P, const uint32_t* __restrict__ U) {
  extern __shared__ uint32_t h[];
  for (uint32_t i = threadIdx.x; i < P.n_levels; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const uint32_t R = P.sc->R_tilde;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < R; i += gridDim.x * blockDim.x) {
    const uint32_t u = U[i];
    if (u < P.n_levels) atomicAdd(&h[u], 1u);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < P.n_levels; i += blockDim.x)
    if (h[i]) atomicAdd(&P.hist[i], h[i]);
}

// --- block-level scans and reductions (wave shuffles + LDS) ----------------
template <int BLOCK>
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total, uint32_t* scratch) {
  constexpr int NW = BLOCK / kWave;
  const uint32_t lane = lane_id(), wid = threadIdx.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, kWave);
    if (lane >= (uint32_t)off) x += y;
  }
  if (lane == kWave - 1) scratch[wid] = x;
  __syncthreads();
  if (wid == 0) {
    uint32_t s = lane < (uint32_t)NW ? scratch[lane] : 0u;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t y = __shfl_up(s, off, kWave);
      if (lane >= (uint32_t)off) s += y;
    }
    if (lane < (uint32_t)NW) scratch[lane] = s;  // inclusive over waves
  }
  __syncthreads();
  const uint32_t before = wid ? scratch[wid - 1] : 0u;
  *total = scratch[NW - 1];
  __syncthreads();
  return before + x - v;
}

template <int BLOCK, typename T>
__device__ T block_sum(T v, T* scratch) {
  constexpr int NW = BLOCK / kWave;
  const uint32_t lane = lane_id(), wid = threadIdx.x / kWave;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  T s = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NW; ++w) s += scratch[w];
  __syncthreads();
  return s;  // valid in thread 0
}

// Nearest-integer copy counts (Sec. II): n_i = fl[U_i] + [u53 < T[U_i]] with
// u53 = (w0 << 21) | (w1 >> 11) from Philox(seed; i, step, 0, RES).
__global__ __launch_bounds__(kBlockCounts) void k_counts(DevPop P, const uint32_t* __restrict__ U,
                                                         uint32_t step) {
  __shared__ uint32_t scratch[kBlockCounts / kWave];
  const uint32_t R = P.sc->R_tilde;
  const uint32_t i = blockIdx.x * kBlockCounts + threadIdx.x;
  uint32_t n = 0, culled = 0;
  if (i < R) {
    const uint32_t u = min(U[i], P.n_levels - 1);
    const Words4 w = philox10(i, step, 0u, kTagRes, (uint32_t)P.seed, (uint32_t)(P.seed >> 32));
    const unsigned long long u53 = ((unsigned long long)w.w[0] << 21) | (w.w[1] >> 11);
    n = P.table_fl[u] + (u53 < P.table_T[u] ? 1u : 0u);
    P.counts[i] = n;
    culled = n == 0;
  }
  const uint32_t s = block_sum<kBlockCounts, uint32_t>(n, scratch);
  const uint32_t c = block_sum<kBlockCounts, uint32_t>(culled, scratch);
  if (threadIdx.x == 0) {
    P.block_sums[blockIdx.x] = s;
    P.block_culled[blockIdx.x] = c;
  }
}

// Exclusive scan of the per-block sums (one workgroup), the new population
// size R~' = sum n_i, and the capacity check.
__global__ __launch_bounds__(1024) void k_scan(DevPop P, uint32_t capacity) {
  __shared__ uint32_t scratch[1024 / kWave];
  __shared__ unsigned long long cull_scratch[1024 / kWave];
  const uint32_t nb = P.n_blocks;
  const uint32_t per = (nb + 1023) / 1024;
  const uint32_t b0 = threadIdx.x * per;
  uint32_t local = 0, cull = 0;
  for (uint32_t b = b0; b < min(b0 + per, nb); ++b) {
    local += P.block_sums[b];
    cull += P.block_culled[b];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan<1024>(local, &total, scratch);
  for (uint32_t b = b0; b < min(b0 + per, nb); ++b) {
    P.block_offsets[b] = run;
    run += P.block_sums[b];
  }
  const unsigned long long ctot =
      block_sum<1024, unsigned long long>((unsigned long long)cull, cull_scratch);
  if (threadIdx.x == 0) {
    P.sc->R_next = total;
    P.sc->err = total > capacity ? 1u : 0u;
    P.sc->n_culled = (uint32_t)ctot;
  }
}

// Offsets and the new-slot -> old-slot map of the order-preserving copy:
// the n_i copies of old slot i take new slots offset_i .. offset_i + n_i - 1.
__global__ __launch_bounds__(kBlockCounts) void k_scatter(DevPop P) {
  __shared__ uint32_t scratch[kBlockCounts / kWave];
  if (P.sc->err) return;
  const uint32_t R = P.sc->R_tilde;
  const uint32_t i = blockIdx.x * kBlockCounts + threadIdx.x;
  const uint32_t n = i < R ? P.counts[i] : 0u;
  uint32_t total;
  const uint32_t excl = block_exclusive_scan<kBlockCounts>(n, &total, scratch);
  if (i < R) {
    const uint32_t off = P.block_offsets[blockIdx.x] + excl;
    P.offsets[i] = off;
    for (uint32_t c = 0; c < n; ++c) P.src[off + c] = i;
  }
}

// Gather (optional) + n_sweeps checkerboard Metropolis sweeps + energy, one
// wavefront per 64-replica tile.  Reads buffer cur, writes buffer cur ^ 1.
template <int LAYOUT, int L>
__global__ __launch_bounds__(64) void k_sweep(DevPop P, SweepParams sp,
                                              const SiteEntry* __restrict__ sites,
                                              const unsigned long long* __restrict__ rowj) {
  constexpr uint32_t N = L * L * L;
  extern __shared__ uint32_t lds[];
  __shared__ unsigned long long thr_of_nu[8];
  const uint32_t tile = blockIdx.x;
  const uint32_t lane = lane_id();
  if (sp.gather && tile == 0 && lane == 0) P.sc->R_tilde = P.sc->R_next;
  const uint32_t Rs = sp.gather ? P.sc->R_next : P.sc->R_tilde;
  if (tile * 64 >= Rs) return;
  if (lane < 8) thr_of_nu[lane] = lane < 3 ? sp.thr[2 - lane] : (1ull << 32);
  const uint32_t j = tile * 64 + lane;
  const bool valid = j < Rs;
  const uint32_t src = valid ? (sp.gather ? P.src[j] : j) : 0u;
  const uint32_t cur = sp.cur, nxt = cur ^ 1u;
  load_tile_gather<LAYOUT>(lds, P.spins[cur], N, src, valid);
  RowCtx c;
  c.lds = lds;
  c.thr_of_nu = thr_of_nu;
  c.h = lane >> 5;
  c.pos = lane & 31u;
  c.slot = j;
  c.k0 = (uint32_t)P.seed;
  c.k1 = (uint32_t)(P.seed >> 32);
  // a draw matters only for a class whose threshold is neither 0 nor 2^32
  c.any_draw = (sp.thr[0] != 0 && sp.thr[0] < (1ull << 32)) ||
               (sp.thr[1] != 0 && sp.thr[1] < (1ull << 32)) ||
               (sp.thr[2] != 0 && sp.thr[2] < (1ull << 32));
  c.d.w[0] = c.d.w[1] = c.d.w[2] = c.d.w[3] = 0u;
  for (uint32_t s = 0; s < sp.n_sweeps; ++s) {
    c.t = sp.t0 + s;
    sweep_colour_rows<L>(c, rowj, 0u);
    sweep_colour_rows<L>(c, rowj, 1u);
  }
  const uint32_t U = tile_energy(lds, sites, N);
  store_tile<LAYOUT>(lds, P.spins[nxt], N, tile);
  if (valid) {
    P.U[nxt][j] = U;
    P.fam[nxt][j] = P.fam[cur][src];
  }
}

// Sum over families of eta^2 (Sec. III.A) from the family labels, which stay
// sorted under the order-preserving copy: each run of equal labels is one
// family; its first slot finds the run's end by binary search.
__global__ __launch_bounds__(256) void k_family(DevPop P, const uint32_t* __restrict__ fam) {
  __shared__ unsigned long long scratch[256 / kWave];
  const uint32_t R = P.sc->R_tilde;
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  unsigned long long sq = 0, nf = 0;
  if (i < R) {
    const uint32_t f = fam[i];
    if (i == 0 || fam[i - 1] != f) {
      uint32_t lo = i + 1, hi = R;  // first index in [i+1, R) with fam != f
      while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (fam[mid] == f) lo = mid + 1;
        else hi = mid;
      }
      const unsigned long long eta = lo - i;
      sq = eta * eta;
      nf = 1;
    }
  }
  const unsigned long long s = block_sum<256, unsigned long long>(sq, scratch);
  const unsigned long long c = block_sum<256, unsigned long long>(nf, scratch);
  if (threadIdx.x == 0) {
    if (s) atomicAdd(&P.sc->sum_eta2, s);
    if (c) atomicAdd(&P.sc->n_families, (uint32_t)c);
  }
}

// Spin-overlap histogram (Sec. II.A): slot i of population A against slot i
// of population B; d = differing sites, bin = (128 (N - d) + N) / (2N).
template <int LAYOUT>
__global__ __launch_bounds__(64) void k_overlap(DevPop A, uint32_t cur_a, DevPop B,
                                                uint32_t cur_b, unsigned long long* hist65) {
  __shared__ uint32_t hb[65];
  const uint32_t tile = blockIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t n = min(A.sc->R_tilde, B.sc->R_tilde);
  if (tile * 64 >= n) return;
  for (uint32_t b = lane; b < 65; b += 64) hb[b] = 0;
  __syncthreads();
  const uint32_t i = tile * 64 + lane;
  const uint32_t N = A.N;
  uint32_t d = 0;
  if (LAYOUT == 2) {
    const unsigned long long* a = static_cast<const unsigned long long*>(A.spins[cur_a]) +
                                  (size_t)tile * N;
    const unsigned long long* b = static_cast<const unsigned long long*>(B.spins[cur_b]) +
                                  (size_t)tile * N;
    for (uint32_t cm = 0; cm < N; ++cm) d += (uint32_t)((a[cm] ^ b[cm]) >> lane) & 1u;
  } else {
    const int8_t* a = static_cast<const int8_t*>(A.spins[cur_a]) + (size_t)tile * N * 64 + lane;
    const int8_t* b = static_cast<const int8_t*>(B.spins[cur_b]) + (size_t)tile * N * 64 + lane;
    for (uint32_t cm = 0; cm < N; ++cm) d += a[64 * (size_t)cm] != b[64 * (size_t)cm];
  }
  if (i < n) atomicAdd(&hb[(128u * (N - d) + N) / (2u * N)], 1u);
  __syncthreads();
  for (uint32_t b = lane; b < 65; b += 64)
    if (hb[b]) atomicAdd(&hist65[b], (unsigned long long)hb[b]);
}

inline uint32_t tiles_of(uint32_t n) { return (n + 63) / 64; }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, stream, p, value, n);
  return hipGetLastError();
}

hipError_t launch_init(const DevPop& P, uint32_t cur, hipStream_t stream) {
  const uint16_t* cm_of_site = P.cm_of_site;
  const size_t lds = (size_t)P.N * 8;
  if (P.layout == 2)
    hipLaunchKernelGGL(k_init<2>, dim3(tiles_of(P.R)), dim3(64), lds, stream, P, cur, cm_of_site);
  else
    hipLaunchKernelGGL(k_init<1>, dim3(tiles_of(P.R)), dim3(64), lds, stream, P, cur, cm_of_site);
  return hipGetLastError();
}

hipError_t launch_energy(const DevPop& P, uint32_t cur, hipStream_t stream) {
  const size_t lds = (size_t)P.N * 8;
  if (P.layout == 2)
    hipLaunchKernelGGL(k_energy<2>, dim3(tiles_of(P.capacity)), dim3(64), lds, stream, P, cur);
  else
    hipLaunchKernelGGL(k_energy<1>, dim3(tiles_of(P.capacity)), dim3(64), lds, stream, P, cur);
  return hipGetLastError();
}

hipError_t launch_hist(const DevPop& P, uint32_t cur, hipStream_t stream) {
  // the caller has zeroed P.hist
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>((P.capacity + 2047) / 2048, 512));
  hipLaunchKernelGGL(k_hist, dim3(grid), dim3(256), (size_t)P.n_levels * 4, stream, P, P.U[cur]);
  return hipGetLastError();
}

hipError_t launch_counts(const DevPop& P, uint32_t cur, uint32_t step, hipStream_t stream) {
  hipLaunchKernelGGL(k_counts, dim3(P.n_blocks), dim3(kBlockCounts), 0, stream, P, P.U[cur], step);
  return hipGetLastError();
}

hipError_t launch_scan(const DevPop& P, hipStream_t stream) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, stream, P, P.cap_limit);
  return hipGetLastError();
}

hipError_t launch_scatter(const DevPop& P, hipStream_t stream) {
  hipLaunchKernelGGL(k_scatter, dim3(P.n_blocks), dim3(kBlockCounts), 0, stream, P);
  return hipGetLastError();
}

template <int LAYOUT>
hipError_t launch_sweep_layout(const DevPop& P, const SweepParams& sp, hipStream_t stream) {
  const size_t lds = (size_t)P.N * 8;
  const dim3 grid(tiles_of(P.capacity)), block(64);
  switch (P.L) {
#define PA_SWEEP_CASE(LL)                                                                     \
  case LL:                                                                                    \
    hipLaunchKernelGGL((k_sweep<LAYOUT, LL>), grid, block, lds, stream, P, sp, P.sites,       \
                       P.rowj);                                                               \
    break;
    PA_SWEEP_CASE(4)
    PA_SWEEP_CASE(6)
    PA_SWEEP_CASE(8)
    PA_SWEEP_CASE(10)
    PA_SWEEP_CASE(12)
    PA_SWEEP_CASE(14)
    PA_SWEEP_CASE(16)
#undef PA_SWEEP_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sweep(const DevPop& P, const SweepParams& sp, hipStream_t stream) {
  return P.layout == 2 ? launch_sweep_layout<2>(P, sp, stream)
                       : launch_sweep_layout<1>(P, sp, stream);
}

hipError_t launch_family(const DevPop& P, uint32_t cur, hipStream_t stream) {
  hipLaunchKernelGGL(k_family, dim3((P.capacity + 255) / 256), dim3(256), 0, stream, P, P.fam[cur]);
  return hipGetLastError();
}

hipError_t launch_overlap(const DevPop& A, uint32_t cur_a, const DevPop& B, uint32_t cur_b,
                          unsigned long long* hist65, hipStream_t stream) {
  const uint32_t grid = tiles_of(std::min(A.capacity, B.capacity));
  if (A.layout == 2)
    hipLaunchKernelGGL(k_overlap<2>, dim3(grid), dim3(64), 0, stream, A, cur_a, B, cur_b, hist65);
  else
    hipLaunchKernelGGL(k_overlap<1>, dim3(grid), dim3(64), 0, stream, A, cur_a, B, cur_b, hist65);
  return hipGetLastError();
}

}  // namespace pa
