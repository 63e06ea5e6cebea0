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
#include <utility>

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
// for a plain copy).  Lanes with valid == false contribute zero bits.  The
// loads are issued eight sites at a time (N = L^3 is a multiple of 8 for even
// L) so that many are in flight before their bits are balloted into LDS.
// Waves that share a tile split its sites: wave `part` of `nparts` takes the
// groups of eight starting at 8 part, 8 (part + nparts), ...
template <int LAYOUT, uint32_t N>
__device__ void load_tile_gather(uint32_t* lds, const void* spins_old, uint32_t src, bool valid,
                                 uint32_t part, uint32_t nparts) {
  constexpr uint32_t B = 8;
  static_assert(N % B == 0, "N must be a multiple of 8");
  const uint32_t lane = lane_id();
  const uint32_t stile = src >> 6;
  const uint32_t pos = LAYOUT == 2 ? (src & 31u) : 0u;
  const uint32_t* w32 = static_cast<const uint32_t*>(spins_old) + (size_t)stile * N * 2 +
                        ((src >> 5) & 1u);
  const int8_t* s8 = static_cast<const int8_t*>(spins_old) + (size_t)stile * N * 64 + (src & 63u);
#pragma unroll 2
  for (uint32_t cm0 = B * part; cm0 < N; cm0 += B * nparts) {
    uint32_t v[B];
#pragma unroll
    for (uint32_t i = 0; i < B; ++i) {
      const uint32_t cm = cm0 + i;
      if (LAYOUT == 2)
        v[i] = w32[2 * (size_t)cm];
      else
        v[i] = (uint32_t)(uint8_t)s8[64 * (size_t)cm];
    }
#pragma unroll
    for (uint32_t i = 0; i < B; ++i) {
      const uint32_t cm = cm0 + i;
      const uint32_t b = LAYOUT == 2 ? bit_of(v[i], pos) : (v[i] >> 7);  // int8: sign bit
      const unsigned long long m = __ballot(valid && b);
      if (lane == 0) {
        lds[2 * cm] = (uint32_t)m;
        lds[2 * cm + 1] = (uint32_t)(m >> 32);
      }
    }
  }
  __syncthreads();
}

template <int LAYOUT>
__device__ void store_tile(const uint32_t* lds, void* spins_new, uint32_t N, uint32_t tile,
                           uint32_t part, uint32_t nparts) {
  const uint32_t lane = lane_id();
  if (LAYOUT == 2) {
    uint2* w = static_cast<uint2*>(spins_new) + (size_t)tile * N;
    for (uint32_t cm = lane + kWave * part; cm < N; cm += kWave * nparts)
      w[cm] = make_uint2(lds[2 * cm], lds[2 * cm + 1]);
  } else {
    int8_t* s8 = static_cast<int8_t*>(spins_new) + (size_t)tile * N * 64 + lane;
    const uint32_t h = lane >> 5, pos = lane & 31u;
    for (uint32_t cm = part; cm < N; cm += nparts)
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

// Philox4x32-10 for the Metropolis draws of one lane.  The counter is
// (slot, t, g, MET): slot is fixed per lane, t and g are wave-uniform.  The
// first round multiplies only slot (a per-lane constant) and g (uniform), so
// round 1 and the slot half of round 2 are computed once per lane; each call
// then costs two XORs for round 2 and four instructions per round for rounds
// 3..10 (two v_mad_u64_u32, two XORs).
struct MetPhilox {
  uint32_t x2, x3;    // round-1 words that depend on slot only
  uint32_t p2hi, p2lo;  // round-2 product of the slot half
  uint32_t k0, k1;    // key (seed)

  __device__ __forceinline__ void init(uint32_t slot, uint32_t key0, uint32_t key1) {
    k0 = key0;
    k1 = key1;
    const uint64_t pa = (uint64_t)0xD2511F53u * slot;
    x2 = (uint32_t)(pa >> 32) ^ kTagMet ^ key1;
    x3 = (uint32_t)pa;
    const uint64_t pb = (uint64_t)0xCD9E8D57u * x2;
    p2hi = (uint32_t)(pb >> 32);
    p2lo = (uint32_t)pb;
  }

  __device__ __forceinline__ Words4 draw(uint32_t t, uint32_t g) const {
    // round 1 (key k): uniform half
    const uint64_t a = (uint64_t)0xCD9E8D57u * g;
    const uint32_t x0 = (uint32_t)(a >> 32) ^ t ^ k0;
    const uint32_t x1 = (uint32_t)a;
    // round 2 (key k + W)
    const uint32_t r2k0 = k0 + 0x9E3779B9u, r2k1 = k1 + 0xBB67AE85u;
    const uint64_t b = (uint64_t)0xD2511F53u * x0;
    uint32_t c0 = p2hi ^ (x1 ^ r2k0);
    uint32_t c1 = p2lo;
    uint32_t c2 = x3 ^ ((uint32_t)(b >> 32) ^ r2k1);
    uint32_t c3 = (uint32_t)b;  // uniform
    uint32_t q0 = k0 + 2u * 0x9E3779B9u, q1 = k1 + 2u * 0xBB67AE85u;
    // round 3: c3 is uniform, fold it into the key word
    {
      const uint64_t pa = (uint64_t)0xD2511F53u * c0;
      const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
      const uint32_t n0 = xor3_s((uint32_t)(pb >> 32), c1, q0);
      const uint32_t n2 = (uint32_t)(pa >> 32) ^ (c3 ^ q1);
      c0 = n0; c1 = (uint32_t)pb; c2 = n2; c3 = (uint32_t)pa;
      q0 += 0x9E3779B9u;
      q1 += 0xBB67AE85u;
    }
#pragma unroll
    for (int r = 3; r < 10; ++r) {
      const uint64_t pa = (uint64_t)0xD2511F53u * c0;
      const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
      const uint32_t n0 = xor3_s((uint32_t)(pb >> 32), c1, q0);
      const uint32_t n2 = xor3_s((uint32_t)(pa >> 32), c3, q1);
      c0 = n0; c1 = (uint32_t)pb; c2 = n2; c3 = (uint32_t)pa;
      q0 += 0x9E3779B9u;
      q1 += 0xBB67AE85u;
    }
    Words4 o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
  }
};

// Row addressing of the LDS tile (the energy of a tile when no sweep runs).
// For even L, the sites of colour c in row rho = y + L z are x = 2q + p,
// q = 0..L/2-1, p = (c + y + z) & 1, with colour-major indices
// c*N/2 + (L/2) rho + q.  Their neighbours of the other colour, in that
// colour's rank order: +x at rank (q + p) mod L/2 and -x at (q + p - 1) mod L/2
// of the same row, and rank q of the rows (y+-1, z) and (y, z+-1).  Per row
// seven base addresses are formed (own row, x row shifted by p, the one
// wrapped x neighbour shared by the last and first site, and the four y/z
// rows); every site reads its words at compile-time offsets from them.
//
// Metropolis test (+-J): nu = number of unsatisfied bonds at the site (own
// bit ^ neighbour bit ^ [J = -1]); flipping changes the energy by
// dE = 12 - 4 nu, and the move is accepted iff its draw is below thr_of_nu[nu]
// (floor(2^32 exp(-beta dE)) for nu <= 2, 2^32 for nu >= 3).  The colour
// passes below sum the post-move energy in the colour-1 pass of the last
// sweep (every bond joins one site of each colour).
struct TileCtx {
  uint32_t* lds;
  const unsigned long long* thr_of_nu;
  uint32_t hoff;   // byte offset of this lane's half word: 4 * (lane >> 5)
  uint32_t pos;    // this lane's bit in its half word
  MetPhilox ph;
  uint32_t t;
  bool any_draw;
  unsigned long long writers;  // lanes 0 and 32: the lanes that apply a site's flips
  uint32_t hshift;             // 8 hoff: shift of a ballot that brings this lane's half down
  // kModelGauss16
  const int8_t* rowk;                  // row couplings (see DevPop)
  uint32_t rowk_stride;
  const uint16_t* gaddr;               // 16 max(he16, 0) of (site, pattern), see DevPop
  // kModelReal
  const unsigned long long* rthr;      // thresholds of (site, pattern) for this sweep
  const uint32_t* rthr32;              // the same, min(thr, 2^32 - 1)
  const long long* rhe;                // half energy changes he of (site, pattern)
};

// Energy accumulator of a pass: 32-bit words for the integer models (the
// sums wrap like the stored words), 64-bit for kModelReal.
template <int M>
struct AccOf {
  using type = uint32_t;
};
template <>
struct AccOf<(int)kModelReal> {
  using type = long long;
};

// A uniform byte offset kept whole in a scalar register.  Added to the lane's
// LDS base it costs one vector add per row pointer; left to the compiler, a
// constant part (the other colour's base) is split off into the access's
// immediate offset, which does not fit the 8-bit fields of ds_read2 and costs
// a second add per pointer.
__device__ __forceinline__ uint32_t whole_s(uint32_t x) {
  asm("" : "+s"(x));
  return x;
}

// Read-only device memory in the constant address space (scalar loads).
typedef const __attribute__((address_space(4))) uint32_t ConstU32;
typedef const __attribute__((address_space(4))) unsigned long long ConstU64;

struct RowAddr {
  const uint32_t* own;
  const uint32_t* x0;    // rank p of the other-colour x row
  const uint32_t* wrap;  // the x neighbour that wraps around
  const uint32_t* py;
  const uint32_t* my;
  const uint32_t* pz;
  const uint32_t* mz;
  unsigned long long j;  // coupling bits of the row (kModelPm)
  ConstU32* krow;        // coupling bytes of the row, 4 per word (kModelGauss16)
  uint32_t cm0;          // colour-major index of the row's first site (kModelReal)
};

template <int L, int M>
__device__ __forceinline__ RowAddr row_addr(const TileCtx& c, const unsigned long long* rowj,
                                            uint32_t colour, uint32_t rho) {
  constexpr uint32_t H = L / 2, N = L * L * L;
  const uint32_t own0 = colour * (N / 2), oth0 = (colour ^ 1u) * (N / 2);
  const uint32_t y = rho % L, z = rho / L;
  const uint32_t yp = y + 1 == (uint32_t)L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
  const uint32_t zp = z + 1 == (uint32_t)L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
  const uint32_t p = (colour + y + z) & 1u;
  const uint32_t ox = oth0 + H * rho;
  const char* base = reinterpret_cast<const char*>(c.lds) + c.hoff;
  RowAddr a;
  a.own = reinterpret_cast<const uint32_t*>(base + whole_s(8 * (own0 + H * rho)));
  a.x0 = reinterpret_cast<const uint32_t*>(base + whole_s(8 * (ox + p)));
  a.wrap = reinterpret_cast<const uint32_t*>(base + whole_s(8 * (ox + (H - 1) * (1u - p))));
  a.py = reinterpret_cast<const uint32_t*>(base + whole_s(8 * (oth0 + H * (yp + L * z))));
  a.my = reinterpret_cast<const uint32_t*>(base + whole_s(8 * (oth0 + H * (ym + L * z))));
  a.pz = reinterpret_cast<const uint32_t*>(base + whole_s(8 * (oth0 + H * (y + L * zp))));
  a.mz = reinterpret_cast<const uint32_t*>(base + whole_s(8 * (oth0 + H * (y + L * zm))));
  // The coupling words are read through the constant address space: the
  // index is uniform and nothing in the kernel writes them, so they arrive in
  // scalar registers and the per-bond masks and bytes are scalar work.
  a.cm0 = own0 + H * rho;
  if constexpr (M == (int)kModelGauss16) {
    a.j = 0;
    a.krow = (const ConstU32*)(c.rowk + (size_t)(colour * L * L + rho) * c.rowk_stride);
  } else if constexpr (M == (int)kModelReal) {
    a.j = 0;
    a.krow = nullptr;
  } else {
    a.j = ((const ConstU64*)rowj)[colour * L * L + rho];
    a.krow = nullptr;
  }
  return a;
}

// The seven words a site reads: its own word and its six neighbours.
struct SiteLoad {
  uint32_t own;
  uint32_t nb[6];
};

template <int L, int Q>
__device__ __forceinline__ SiteLoad load_site_words(const RowAddr& a) {
  constexpr int H = L / 2;
  SiteLoad w;
  w.own = a.own[2 * Q];
  w.nb[0] = Q < H - 1 ? a.x0[2 * Q] : a.wrap[0];
  w.nb[1] = Q > 0 ? a.x0[2 * (Q - 1)] : a.wrap[0];
  w.nb[2] = a.py[2 * Q];
  w.nb[3] = a.my[2 * Q];
  w.nb[4] = a.pz[2 * Q];
  w.nb[5] = a.mz[2 * Q];
  return w;
}

// Coupling k (in quanta 1/16) of site Q of a row to its neighbour K: a
// sign-extended byte of the row's words (uniform: scalar registers).
template <int Q, int K>
__device__ __forceinline__ int32_t row_k(const RowAddr& a) {
  constexpr int b = 6 * Q + K;
  const uint32_t w = a.krow[b / 4];
  return (int32_t)(w << (24 - 8 * (b % 4))) >> 24;
}

// Pattern y of a site for this lane: bit k set iff neighbour k's spin differs
// from the site's own (k in the order +x,-x,+y,-y,+z,-z).
__device__ __forceinline__ uint32_t real_pattern(const TileCtx& c, const SiteLoad& w) {
  uint32_t y = __builtin_amdgcn_ubfe(w.nb[0] ^ w.own, c.pos, 1);
#pragma unroll
  for (int k = 1; k < 6; ++k) y |= __builtin_amdgcn_ubfe(w.nb[k] ^ w.own, c.pos, 1) << k;
  return y;
}

// ---------------------------------------------------------------------------
// +-J colour pass in two phases.  The bond arithmetic of a site is the same
// for its 64 replicas up to their bits, so it is done once per site on whole
// 32-bit words: phase 1 gives each lane one site (lane = site), forms the six
// words x_k = neighbour ^ own ^ J mask (bit r set iff bond k of replica r is
// unsatisfied), adds them bitwise with two full adders and a half adder into
// three bit planes, nu = p0 + 2 p1 + 4 p2 per replica, and spreads the planes
// into one byte per replica holding 8 nu, the byte address of the replica's
// threshold.  Phase 2 returns to lane = replica: each lane reads its byte and
// applies the Metropolis test with the same draw as before.  nu, the draws and
// the test are unchanged, so every result is too.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xor3_v(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// bitwise majority of three words (v_bitop3_b32 truth table 0xe8)
__device__ __forceinline__ uint32_t maj3_v(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xe8" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

struct NuPlanes {
  uint32_t p0, p1, p2;
};

// nu of 32 replicas as bit planes: x0 + .. + x5 = (s1 + 2 c1) + (s2 + 2 c2)
// = p0 + 2 (c1 + c2 + c3) with p0 = s1 ^ s2, c3 = s1 & s2, and c1 + c2 + c3 =
// p1 + 2 p2 (their XOR and majority).
__device__ __forceinline__ NuPlanes nu_planes(uint32_t own, const uint32_t (&nb)[6],
                                              const uint32_t (&jm)[6]) {
  uint32_t x[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) x[k] = xor3_v(nb[k], own, jm[k]);
  const uint32_t s1 = xor3_v(x[0], x[1], x[2]), c1 = maj3_v(x[0], x[1], x[2]);
  const uint32_t s2 = xor3_v(x[3], x[4], x[5]), c2 = maj3_v(x[3], x[4], x[5]);
  const uint32_t c3 = s1 & s2;
  NuPlanes r;
  r.p0 = s1 ^ s2;
  r.p1 = xor3_v(c1, c2, c3);
  r.p2 = maj3_v(c1, c2, c3);
  return r;
}

// Word j (j = 0..7) of a half's 32 bytes: byte m holds 8 nu of the replica at
// bit j + 8m of the planes.  With p1 rotated left by 1 and p2 by 2 (once per
// half), the bits that word j needs sit at positions j, j + 1, j + 2 (mod 8)
// of p0, p1', p2' and never overlap: three masked merges collect them and one
// rotation right by j - 3 moves bit j + 8m of p0 to 8m + 3, of p1 to 8m + 4
// and of p2 to 8m + 5.  The replica at bit b of a half therefore finds its
// byte at 4 (b & 7) + (b >> 3) (plane_byte below).
__device__ __forceinline__ uint32_t rotr32(uint32_t x, uint32_t s) {
  return __builtin_amdgcn_alignbit(x, x, s);
}

struct NuPlanesRot {
  uint32_t p0, p1r, p2r;  // p0, p1 rotated left by 1, p2 rotated left by 2
};

__device__ __forceinline__ NuPlanesRot rot_planes(const NuPlanes& p) {
  NuPlanesRot r;
  r.p0 = p.p0;
  r.p1r = rotr32(p.p1, 31);
  r.p2r = rotr32(p.p2, 30);
  return r;
}

template <int J>
__device__ __forceinline__ uint32_t nu8_word(const NuPlanesRot& p) {
  constexpr uint32_t m = 0x01010101u << J;
  constexpr uint32_t m1 = (m << 1) | (m >> 31), m2 = (m << 2) | (m >> 30);
  const uint32_t t = (p.p0 & m) | (p.p1r & m1) | (p.p2r & m2);
  return rotr32(t, (J - 3) & 31);
}

// The two-plane form of the same spread for the class c = min(nu, 3) of a
// replica (c0 = p0 | p2, c1 = p1 | p2, c1 rotated left by 1 once per half):
// word J, byte m holds 8 c of the replica at bit J + 8m, at bits 3 and 4.
template <int J>
__device__ __forceinline__ uint32_t cls8_word(uint32_t c0, uint32_t c1r) {
  constexpr uint32_t m = 0x01010101u << J;
  constexpr uint32_t m1 = (m << 1) | (m >> 31);
  return rotr32((c0 & m) | (c1r & m1), (J - 3) & 31);
}

// byte of replica r (lane r) within a site's 64 bytes, before the rotation below
__device__ __forceinline__ uint32_t plane_byte(uint32_t r) {
  return (r & 32u) + 4u * (r & 7u) + ((r >> 3) & 3u);
}

// The +-J colour pass gives each wave one contiguous range of the colour's
// sites (same-colour sites are independent, and a range that starts on a
// multiple of 4 holds whole Philox groups), taken 64 sites (one per lane in
// phase 1) at a time.  W sites per wave: an even share rounded up to whole
// groups; the last wave's range is shorter.
template <int L, int SPLIT>
constexpr uint32_t wave_sites() {
  return ((uint32_t)(L * L * L / 2 + SPLIT - 1) / SPLIT + 3u) / 4u * 4u;
}

// Plane area of a wave: entry e (the e-th site of a 64-site chunk) is 64
// bytes at 64 e, the replicas' bytes in four 16-byte slots: the 16 bytes a
// phase-1 lane forms as words 4j .. 4j + 3 go to slot (j + rot(e)) & 3.  With
// rot(e) = ((e >> 1) + (e >> 3)) & 3, each 16-byte store of phase 1 puts the
// 16 (or 8) lanes the LDS serves together in different banks, for 64 banks
// of 4 bytes and for 32; unrotated, lanes 64 bytes apart share banks.
__host__ __device__ constexpr uint32_t plane_rot(uint32_t e) { return ((e >> 1) + (e >> 3)) & 3u; }

// Phase 1 for a chunk of n <= 64 sites from colour-major index cm0: lane e < n
// takes site cm0 + e, reads its six neighbours' words (absolute LDS addresses
// from the site table) and its own, forms the bit planes of nu for both
// 32-replica halves and writes its plane entry.
//
// FAST (every move that raises the energy has a threshold below 2^32): the
// replicas with nu >= 3, whose move does not raise the energy and is always
// taken, are flipped here, in the site's word, and the bytes hold 8 min(nu, 3).
// Phase 2 then reads the low 32-bit word of the threshold table at that byte:
// thr(nu) for nu <= 2, and 0 (never, the move is done) for nu >= 3.  Only this
// wave writes the words of its own sites during the pass, and phase 2 does not
// read them, so the early flip changes nothing but the order of the XORs.
// Otherwise the bytes hold 8 nu (the 64-bit table's byte address).
template <bool FAST>
__device__ __forceinline__ void plane_chunk(const TileCtx& c, const PlaneSite* __restrict__ sites,
                                            uint32_t cm0, uint32_t n, uint32_t lane,
                                            char* planes) {
  if (lane < n) {
    const uint32_t cm = cm0 + lane;
    const uint4 e0 = reinterpret_cast<const uint4*>(sites)[2 * cm];
    const uint4 e1 = reinterpret_cast<const uint4*>(sites)[2 * cm + 1];
    const uint32_t nb8[6] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y};
    const uint32_t jneg = e1.z;
    uint2* w = reinterpret_cast<uint2*>(c.lds);
    // LDS address 0: the table's addresses are absolute (the kernel has
    // checked that the tile image starts at kTileLdsBase)
    const char* lds0 = reinterpret_cast<const char*>(c.thr_of_nu);
    const uint2 o = w[cm];
    uint32_t lo[6], hi[6], jm[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const uint2 v = *reinterpret_cast<const uint2*>(lds0 + nb8[k]);
      lo[k] = v.x;
      hi[k] = v.y;
      jm[k] = (uint32_t)((int32_t)(jneg << (31 - k)) >> 31);
    }
    const NuPlanes pa = nu_planes(o.x, lo, jm);
    const NuPlanes pb = nu_planes(o.y, hi, jm);
    uint4 q[4];
    if constexpr (FAST) {
      // nu >= 3: p2 | (p1 & p0); flipped now
      w[cm] = make_uint2(o.x ^ (pa.p2 | (pa.p1 & pa.p0)), o.y ^ (pb.p2 | (pb.p1 & pb.p0)));
      const uint32_t a0 = pa.p0 | pa.p2, a1 = rotr32(pa.p1 | pa.p2, 31);
      const uint32_t b0 = pb.p0 | pb.p2, b1 = rotr32(pb.p1 | pb.p2, 31);
      q[0] = make_uint4(cls8_word<0>(a0, a1), cls8_word<1>(a0, a1), cls8_word<2>(a0, a1),
                        cls8_word<3>(a0, a1));
      q[1] = make_uint4(cls8_word<4>(a0, a1), cls8_word<5>(a0, a1), cls8_word<6>(a0, a1),
                        cls8_word<7>(a0, a1));
      q[2] = make_uint4(cls8_word<0>(b0, b1), cls8_word<1>(b0, b1), cls8_word<2>(b0, b1),
                        cls8_word<3>(b0, b1));
      q[3] = make_uint4(cls8_word<4>(b0, b1), cls8_word<5>(b0, b1), cls8_word<6>(b0, b1),
                        cls8_word<7>(b0, b1));
    } else {
      const NuPlanesRot a = rot_planes(pa);
      const NuPlanesRot b = rot_planes(pb);
      q[0] = make_uint4(nu8_word<0>(a), nu8_word<1>(a), nu8_word<2>(a), nu8_word<3>(a));
      q[1] = make_uint4(nu8_word<4>(a), nu8_word<5>(a), nu8_word<6>(a), nu8_word<7>(a));
      q[2] = make_uint4(nu8_word<0>(b), nu8_word<1>(b), nu8_word<2>(b), nu8_word<3>(b));
      q[3] = make_uint4(nu8_word<4>(b), nu8_word<5>(b), nu8_word<6>(b), nu8_word<7>(b));
    }
    char* const entry = planes + 64 * lane;
    const uint32_t rot = plane_rot(lane);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
      *reinterpret_cast<uint4*>(entry + 16 * ((j + rot) & 3u)) = q[j];
  }
}

// XOR of data into the LDS word at addr + OFF by the two lanes in `writers`
// (lanes 0 and 32: one per 32-replica half of a site word), under an exec
// mask set and restored in the same statement.  Written as a branch around an
// atomic, the flip would split the unrolled sites into basic blocks, and the
// compiler would then mask every prefetched threshold byte again.  All 64
// lanes are active wherever this is called, so exec is set to `writers`
// outright: only s_mov_b64 touches it, which leaves SCC alone (the compiler
// may hold a branch condition in SCC across this statement; s_and_saveexec
// would overwrite it).
template <int OFF>
__device__ __forceinline__ void lds_xor_two_lanes(const char* addr, uint32_t data,
                                                  unsigned long long writers) {
  unsigned long long saved;
  const uint32_t a = (uint32_t)(uintptr_t)addr;
  asm volatile(
      "s_mov_b64 %0, exec\n\t"
      "s_mov_b64 exec, %3\n\t"
      "ds_xor_b32 %1, %2 offset:%4\n\t"
      "s_mov_b64 exec, %0"
      : "=&s"(saved)
      : "v"(a), "v"(data), "s"(writers), "i"(OFF)
      : "memory");
}

// The lane's byte of entry E of a chunk: one of four per-lane addresses (by
// the entry's rotation) plus 64 E, a constant offset of the instruction.
struct PlaneReads {
  const uint8_t* at[4];  // the lane's byte for entries of rotation 0..3, entry 0
};

template <int E>
__device__ __forceinline__ uint32_t plane_read(const PlaneReads& pr) {
  return (uint32_t)pr.at[plane_rot(E)][64 * E];
}

// Phase 2 for sites E.. of a chunk of n sites (n uniform): the Metropolis
// test of this lane's replica at each site, and the flip.  A new Philox call
// starts every fourth site, whether or not a draw can matter (a threshold of
// 0 or 2^32 decides without it), so that each group of four sites is one
// basic block; the chunk ends at the first group at or past n.  The byte of
// site E + 1 of the same group is read before site E is updated (the plane
// area is not written in this phase), so its LDS latency overlaps the update.
//
// FAST: the byte is 8 min(nu, 3) and the threshold the table's low 32-bit
// word (see plane_chunk): one 32-bit compare.  Otherwise the byte is 8 nu and
// the threshold the whole 64-bit entry (2^32: always taken); with ACCUM the
// lane also sums its replica's post-move nu.
template <int E, bool FAST, bool ACCUM>
__device__ __forceinline__ void chunk_sites(const TileCtx& c, const char* ownb,
                                            const PlaneReads& pr, uint32_t g0, uint32_t n,
                                            Words4& d, uint32_t& usum, uint32_t a8) {
  if constexpr (E % 4 == 0) {
    if ((uint32_t)E >= n) return;
    a8 = plane_read<E>(pr);
    d = c.ph.draw(c.t, g0 + (uint32_t)(E / 4));
  }
  uint32_t nx = 0;
  if constexpr (E % 4 != 3) nx = plane_read<E + 1>(pr);
  bool acc;
  if constexpr (FAST) {
    const uint32_t thr =
        *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(c.thr_of_nu) + a8);
    acc = d.w[E % 4] < thr;
  } else {
    const unsigned long long thr = *reinterpret_cast<const unsigned long long*>(
        reinterpret_cast<const char*>(c.thr_of_nu) + a8);
    acc = (unsigned long long)d.w[E % 4] < thr;
    if (ACCUM) {
      const uint32_t nu = a8 >> 3;
      usum += acc ? 6u - nu : nu;
    }
  }
  // this lane's half of the ballot: one 64-bit shift of the scalar mask
  const uint32_t fh = (uint32_t)(__ballot(acc) >> c.hshift);
  lds_xor_two_lanes<8 * E>(ownb, fh, c.writers);
  if constexpr (E + 1 < 64) chunk_sites<E + 1, FAST, ACCUM>(c, ownb, pr, g0, n, d, usum, nx);
}

// One +-J colour pass of this wave over its range of wave_sites() sites, a
// 64-site chunk at a time: phase 1 for the chunk, then phase 2.  The wave's
// plane area holds one chunk.  FAST passes skip phase 2 when no move that
// raises the energy can be taken (every such threshold 0): phase 1 has done
// all the flips.  The pass ends with a workgroup barrier, so the next colour
// sees every flip.
template <int L, int SPLIT, bool FAST, bool ACCUM>
__device__ uint32_t sweep_colour_planes(const TileCtx& c, const PlaneSite* __restrict__ sites,
                                        uint32_t colour, uint32_t part, char* planes,
                                        const PlaneReads& pr, uint32_t lane) {
  static_assert(!(FAST && ACCUM), "the energy is summed by the 64-bit form of the pass");
  constexpr uint32_t N = L * L * L, HALF = N / 2, W = wave_sites<L, SPLIT>();
  const uint32_t own0 = colour * HALF;
  const uint32_t first = part * W;
  const uint32_t last = min(first + W, HALF);
  uint32_t usum = 0;
  Words4 d;
  d.w[0] = d.w[1] = d.w[2] = d.w[3] = 0u;
  const char* const own_h = reinterpret_cast<const char*>(c.lds) + c.hoff;
  const bool phase2 = !FAST || c.any_draw;
  for (uint32_t s0 = first; s0 < last; s0 += 64) {
    const uint32_t n = __builtin_amdgcn_readfirstlane(min(64u, last - s0));
    const uint32_t cm0 = own0 + s0;
    plane_chunk<FAST>(c, sites, cm0, n, lane, planes);
    __builtin_amdgcn_wave_barrier();
    if (phase2) {
      const char* ownb = own_h + whole_s(8 * cm0);
      chunk_sites<0, FAST, ACCUM>(c, ownb, pr, cm0 >> 2, n, d, usum, 0u);
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  return usum;
}

// ---------------------------------------------------------------------------
// Gaussian colour pass (quantised and real couplings) in the same two phases.
// The threshold of a move depends on the site and on the pattern y of its six
// "neighbour differs" bits (bit k: s_i != s_k, k in the order +x,-x,+y,-y,
// +z,-z).  Phase 1 (lane = site) forms the six words x_k = neighbour ^ own of
// 32 replicas each and spreads them into one byte per replica holding y << B;
// phase 2 (lane = replica) reads its byte and looks up the site's threshold
// for it: for real couplings min(thr[cm][y], 2^32 - 1) of the sweep's beta (4
// bytes, byte offset 4 y, B = 2; see pattern_groups for the draw 2^32 - 1),
// for quantised ones the entry a[cm][y] = 16 max(he16, 0)
// of a fixed table (2 bytes, byte offset 2 y, B = 1), the byte address of the
// dE16 = 2 he16 threshold in the workgroup's LDS copy of the dE16 table.  The draws,
// the thresholds and the test are those of the one-site-at-a-time form.
// ---------------------------------------------------------------------------

__device__ __forceinline__ constexpr uint32_t rotl_c(uint32_t m, int k) {
  return k == 0 ? m : (m << k) | (m >> (32 - k));
}

// The pattern byte of a replica holds y << B: the byte offset of its entry
// in the site's table row (quantised couplings: 2-byte entries, B = 1; real
// couplings: 4-byte thresholds, B = 2).
template <int M>
constexpr int pattern_shift() {
  return M == (int)kModelReal ? 2 : 1;
}

// Word J (J = 0..7) of a half's 32 bytes: byte m holds y << B of the replica
// at bit J + 8m.  With plane k rotated left by k (once per half, xr[k]), the
// bit that word J needs from plane k sits at J + k + 8m (mod 32): the six
// masked merges never overlap (k < 8), and one rotation right by J - B moves
// it to 8m + B + k.  The replica at bit b of a half finds its byte where the
// +-J pass puts it (plane_byte).
template <int J, int B>
__device__ __forceinline__ uint32_t pattern_word(const uint32_t (&xr)[6]) {
  constexpr uint32_t m = 0x01010101u << J;
  uint32_t t = xr[0] & m;
#pragma unroll
  for (int k = 1; k < 6; ++k) t = (xr[k] & rotl_c(m, k)) | t;
  return J == B ? t : rotr32(t, (uint32_t)(J - B) & 31u);
}

// Phase 1 of the Gaussian pass for a chunk of n <= 64 sites from colour-major
// index cm0 (see plane_chunk: same site table, same entry layout).  Lanes past
// n take site n - 1 again, so that every entry of the area holds a pattern of
// a site of the chunk (phase 2 reads one group past the chunk's end ahead).
template <int M>
__device__ __forceinline__ void pattern_chunk(const TileCtx& c, const PlaneSite* __restrict__ sites,
                                              uint32_t cm0, uint32_t n, uint32_t lane,
                                              char* planes) {
  {
    const uint32_t cm = cm0 + min(lane, n - 1u);
    const uint4 e0 = reinterpret_cast<const uint4*>(sites)[2 * cm];
    const uint2 e1 = reinterpret_cast<const uint2*>(sites)[4 * cm + 2];
    const uint32_t nb8[6] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y};
    const uint2* w = reinterpret_cast<const uint2*>(c.lds);
    const char* lds0 = reinterpret_cast<const char*>(c.thr_of_nu);  // LDS address 0
    const uint2 o = w[cm];
    uint32_t xa[6], xb[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const uint2 v = *reinterpret_cast<const uint2*>(lds0 + nb8[k]);
      xa[k] = k == 0 ? v.x ^ o.x : rotr32(v.x ^ o.x, 32u - (uint32_t)k);
      xb[k] = k == 0 ? v.y ^ o.y : rotr32(v.y ^ o.y, 32u - (uint32_t)k);
    }
    constexpr int B = pattern_shift<M>();
    uint4 q[4];
    q[0] = make_uint4(pattern_word<0, B>(xa), pattern_word<1, B>(xa), pattern_word<2, B>(xa),
                      pattern_word<3, B>(xa));
    q[1] = make_uint4(pattern_word<4, B>(xa), pattern_word<5, B>(xa), pattern_word<6, B>(xa),
                      pattern_word<7, B>(xa));
    q[2] = make_uint4(pattern_word<0, B>(xb), pattern_word<1, B>(xb), pattern_word<2, B>(xb),
                      pattern_word<3, B>(xb));
    q[3] = make_uint4(pattern_word<4, B>(xb), pattern_word<5, B>(xb), pattern_word<6, B>(xb),
                      pattern_word<7, B>(xb));
    char* const entry = planes + 64 * lane;
    const uint32_t rot = plane_rot(lane);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
      *reinterpret_cast<uint4*>(entry + 16 * ((j + rot) & 3u)) = q[j];
  }
}

// Global memory (vector loads with a uniform 64-bit base and a 32-bit lane
// offset).
typedef const __attribute__((address_space(1))) char GlobalChar;

// The threshold of this lane's move at site cm from its byte b = y << B, in two
// stages so that a group's reads can be issued ahead: pattern_ref reads the
// site's table entry (real couplings: min(thr, 2^32 - 1); quantised: the LDS
// byte offset of the dE16 threshold) and pattern_thr finishes it (quantised:
// the read of the LDS dE16 table, at byte address GT).
template <int M>
struct PatternRef {
  using type = uint32_t;
};

// Bytes per site of the table pattern_ref reads, and its first row.
template <int M>
constexpr uint32_t pattern_row_bytes() {
  return M == (int)kModelReal ? kRealPatterns * 4 : kRealPatterns * 2;
}
template <int M>
__device__ __forceinline__ GlobalChar* pattern_table(const TileCtx& c) {
  if constexpr (M == (int)kModelReal)
    return (GlobalChar*)c.rthr32;
  else
    return (GlobalChar*)c.gaddr;
}

// row: the site's row of the table (a uniform address), b: the lane's byte.
template <int M>
__device__ __forceinline__ typename PatternRef<M>::type pattern_ref(GlobalChar* row, uint32_t b) {
  // (a plain 32-bit lane offset: left to itself, the compiler masks the byte
  // again and forms a 64-bit address per lane)
  asm("" : "+v"(b));
  if constexpr (M == (int)kModelReal)
    return *(const __attribute__((address_space(1))) uint32_t*)(row + b);
  else
    return *(const __attribute__((address_space(1))) uint16_t*)(row + b);
}

template <int M, uint32_t GT>
__device__ __forceinline__ unsigned long long pattern_thr(const TileCtx& c,
                                                         typename PatternRef<M>::type r) {
  if constexpr (M == (int)kModelReal) {
    return r;
  } else {
    return *reinterpret_cast<const unsigned long long*>(
        reinterpret_cast<const char*>(c.thr_of_nu) + GT + r);
  }
}

// The site's bond energy he (see kModelReal) for this lane's pattern: the
// site contributes -he before its move and +he after it.  Quantised
// couplings keep only 16 max(he16, 0) per pattern; he16(y ^ 63) = -he16(y)
// (every bit of the pattern inverted), so he16 = (a[y] - a[y ^ 63]) / 16.
template <int M>
__device__ __forceinline__ typename AccOf<M>::type pattern_he(const TileCtx& c, uint32_t cm,
                                                             uint32_t b) {
  if constexpr (M == (int)kModelReal) {
    GlobalChar* row = (GlobalChar*)(c.rhe + (size_t)cm * kRealPatterns);
    return *(const __attribute__((address_space(1))) long long*)(row + 2u * b);
  } else {
    GlobalChar* row = (GlobalChar*)(c.gaddr + (size_t)cm * kRealPatterns);
    const int32_t a = *(const __attribute__((address_space(1))) uint16_t*)(row + b);
    const int32_t an = *(const __attribute__((address_space(1))) uint16_t*)(row + (b ^ 126u));
    return (uint32_t)((a - an) >> 4);
  }
}

// The flips of site E of a chunk (taken: the wave's mask of accepted moves),
// and with ACCUM this lane's share of the energy.
template <int M, int E, bool ACCUM>
__device__ __forceinline__ void pattern_site(const TileCtx& c, const char* ownb, uint32_t cm0,
                                             uint32_t b, unsigned long long taken,
                                             typename AccOf<M>::type& esum) {
  if (ACCUM) {
    const bool acc = ((taken >> lane_id()) & 1ull) != 0ull;
    const typename AccOf<M>::type he = pattern_he<M>(c, cm0 + E, b);
    esum += acc ? he : -he;
  }
  const uint32_t fh = (uint32_t)(taken >> c.hshift);
  lds_xor_two_lanes<8 * E>(ownb, fh, c.writers);
}

// The bytes of group G of a chunk and their table entries (pattern_ref).
// rows: the chunk's first row.  A group past the chunk's end (n) reads bytes
// of the chunk's last site and the rows of the sites after it (the tables
// have kPatternPadRows rows to spare); its entries are never used.
template <int M, int G>
__device__ __forceinline__ void group_refs(GlobalChar* rows, const PlaneReads& pr,
                                           uint32_t (&b)[4],
                                           typename PatternRef<M>::type (&r)[4]) {
  constexpr uint32_t RB = pattern_row_bytes<M>();
  b[0] = plane_read<4 * G>(pr);
  b[1] = plane_read<4 * G + 1>(pr);
  b[2] = plane_read<4 * G + 2>(pr);
  b[3] = plane_read<4 * G + 3>(pr);
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = pattern_ref<M>(rows + (4 * G + i) * RB, b[i]);
}

// Phase 2 of the Gaussian pass for the four sites of group G of a chunk and
// the groups after it (n uniform: the chunk ends at the first group at or past
// n).  The table entries of group G (b, r) were read one group earlier; this
// group reads those of group G + 1 before its own Philox call and tests, so
// that the latency of the dependent reads (byte, table entry, and for
// quantised couplings the LDS threshold) overlaps a group's work.  The plane
// area and the tables are not written in this phase.
template <int M, uint32_t GT, int G, bool ACCUM>
__device__ __forceinline__ void pattern_groups(const TileCtx& c, const char* ownb,
                                               const PlaneReads& pr, GlobalChar* rows,
                                               uint32_t cm0, uint32_t n, const uint32_t (&b)[4],
                                               const typename PatternRef<M>::type (&r)[4],
                                               typename AccOf<M>::type& esum) {
  if ((uint32_t)(4 * G) >= n) return;
  constexpr uint32_t RB = pattern_row_bytes<M>();
  uint32_t bn[4];
  typename PatternRef<M>::type rn[4];
  if constexpr (G + 1 < 16) {
    bn[0] = plane_read<4 * G + 4>(pr);
    bn[1] = plane_read<4 * G + 5>(pr);
    bn[2] = plane_read<4 * G + 6>(pr);
    bn[3] = plane_read<4 * G + 7>(pr);
  }
  unsigned long long thr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) thr[i] = pattern_thr<M, GT>(c, r[i]);
  if constexpr (G + 1 < 16) {
    // the next group's first row as a base of its own in scalar registers:
    // the four reads then take 12-bit immediate offsets from it (left to
    // itself, the compiler runs out of offset range and forms 64-bit
    // addresses per lane)
    GlobalChar* rg = rows + (4 * G + 4) * RB;
    asm("" : "+s"(rg));
#pragma unroll
    for (int i = 0; i < 4; ++i) rn[i] = pattern_ref<M>(rg + i * RB, bn[i]);
  }
  const Words4 d = c.ph.draw(c.t, (cm0 >> 2) + (uint32_t)G);
  // the wave's masks of accepted moves at the group's four sites
  unsigned long long taken[4];
  if constexpr (M == (int)kModelReal) {
    // The 32-bit entry min(thr, 2^32 - 1) decides every draw as thr does but
    // one: for the draw 2^32 - 1 the thresholds 2^32 (taken) and 2^32 - 1 (not
    // taken) share the entry.  Lanes with that draw (a group of a wave has one
    // in about 2^24) read the site's exact threshold.
#pragma unroll
    for (int i = 0; i < 4; ++i) taken[i] = __ballot(d.w[i] < r[i]);
    const uint32_t mx = max(max(d.w[0], d.w[1]), max(d.w[2], d.w[3]));
    if (__builtin_expect(__ballot(mx == 0xFFFFFFFFu) != 0ull, 0)) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool top = d.w[i] == 0xFFFFFFFFu;
        bool exact = false;
        if (top)
          exact = *(const __attribute__((address_space(1))) unsigned long long*)(
                      (GlobalChar*)(c.rthr + (size_t)(cm0 + 4 * G + i) * kRealPatterns) +
                      2u * b[i]) > 0xFFFFFFFFull;
        taken[i] = (taken[i] & ~__ballot(top)) | __ballot(exact);
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) taken[i] = __ballot((unsigned long long)d.w[i] < thr[i]);
  }
  pattern_site<M, 4 * G, ACCUM>(c, ownb, cm0, b[0], taken[0], esum);
  pattern_site<M, 4 * G + 1, ACCUM>(c, ownb, cm0, b[1], taken[1], esum);
  pattern_site<M, 4 * G + 2, ACCUM>(c, ownb, cm0, b[2], taken[2], esum);
  pattern_site<M, 4 * G + 3, ACCUM>(c, ownb, cm0, b[3], taken[3], esum);
  if constexpr (G + 1 < 16)
    pattern_groups<M, GT, G + 1, ACCUM>(c, ownb, pr, rows, cm0, n, bn, rn, esum);
}

// One Gaussian colour pass of this wave over its range of wave_sites() sites,
// a 64-site chunk at a time (see sweep_colour_planes).
template <int L, int SPLIT, int M, bool ACCUM>
__device__ typename AccOf<M>::type sweep_colour_patterns(const TileCtx& c,
                                                         const PlaneSite* __restrict__ sites,
                                                         uint32_t colour, uint32_t part,
                                                         char* planes, const PlaneReads& pr,
                                                         uint32_t lane) {
  constexpr uint32_t N = L * L * L, HALF = N / 2, W = wave_sites<L, SPLIT>();
  const uint32_t own0 = colour * HALF;
  const uint32_t first = part * W;
  const uint32_t last = min(first + W, HALF);
  typename AccOf<M>::type esum = 0;
  const char* const own_h = reinterpret_cast<const char*>(c.lds) + c.hoff;
  for (uint32_t s0 = first; s0 < last; s0 += 64) {
    const uint32_t n = __builtin_amdgcn_readfirstlane(min(64u, last - s0));
    const uint32_t cm0 = __builtin_amdgcn_readfirstlane(own0 + s0);
    pattern_chunk<M>(c, sites, cm0, n, lane, planes);
    __builtin_amdgcn_wave_barrier();
    const char* ownb = own_h + whole_s(8 * cm0);
    GlobalChar* const rows = pattern_table<M>(c) + (size_t)cm0 * pattern_row_bytes<M>();
    uint32_t b[4];
    typename PatternRef<M>::type r[4];
    group_refs<M, 0>(rows, pr, b, r);
    pattern_groups<M, kTileLdsBase + 8 * N + kPlaneAreaBytes * SPLIT, 0, ACCUM>(c, ownb, pr, rows,
                                                                             cm0, n, b, r, esum);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  return esum;
}

// One row's share of tile_energy_rows, sites Q.. of the row.
template <int L, int M, int Q>
__device__ __forceinline__ void tile_energy_row(const TileCtx& c, const RowAddr& a,
                                                typename AccOf<M>::type& U) {
  constexpr int H = L / 2;
  const SiteLoad w = load_site_words<L, Q>(a);
  if constexpr (M == (int)kModelReal) {
    U -= c.rhe[(a.cm0 + Q) * kRealPatterns + real_pattern(c, w)];
  } else if constexpr (M == (int)kModelGauss16) {
    const int32_t k0 = row_k<Q, 0>(a), k1 = row_k<Q, 1>(a), k2 = row_k<Q, 2>(a);
    const int32_t k3 = row_k<Q, 3>(a), k4 = row_k<Q, 4>(a), k5 = row_k<Q, 5>(a);
    const int32_t csum = k0 + k1 + k2 + k3 + k4 + k5;
    const int32_t acc = (int32_t)__builtin_amdgcn_ubfe(w.nb[0] ^ w.own, c.pos, 1) * k0 +
                        (int32_t)__builtin_amdgcn_ubfe(w.nb[1] ^ w.own, c.pos, 1) * k1 +
                        (int32_t)__builtin_amdgcn_ubfe(w.nb[2] ^ w.own, c.pos, 1) * k2 +
                        (int32_t)__builtin_amdgcn_ubfe(w.nb[3] ^ w.own, c.pos, 1) * k3 +
                        (int32_t)__builtin_amdgcn_ubfe(w.nb[4] ^ w.own, c.pos, 1) * k4 +
                        (int32_t)__builtin_amdgcn_ubfe(w.nb[5] ^ w.own, c.pos, 1) * k5;
    U += (uint32_t)(2 * acc - csum);
  } else {
    const uint32_t jlo = (uint32_t)a.j, jhi = (uint32_t)(a.j >> 32);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int bit = 6 * Q + k;
      const uint32_t jm = bit < 32 ? (uint32_t)((int32_t)(jlo << (31 - bit)) >> 31)
                                   : (uint32_t)((int32_t)(jhi << (63 - bit)) >> 31);
      U += __builtin_amdgcn_ubfe(xor3_s(w.nb[k], w.own, jm), c.pos, 1);
    }
  }
  if constexpr (Q + 1 < H) tile_energy_row<L, M, Q + 1>(c, a, U);
}

// Energy of the tile when no sweep ran: sum over colour-0 sites of nu (every
// bond joins one site of each colour); for kModelGauss16 the sum over colour-0
// sites of -sum_k k_k s_i s_k = 2 acc - csum with csum = sum_k k_k and acc =
// sum_k k_k [s_i != s_k], i.e. E16; for kModelReal the sum of -he.
template <int L, int M>
__device__ typename AccOf<M>::type tile_energy_rows(const TileCtx& c,
                                                    const unsigned long long* rowj, uint32_t part,
                                                    uint32_t nparts) {
  constexpr uint32_t ROWS = L * L;
  typename AccOf<M>::type U = 0;
  for (uint32_t rho = part; rho < ROWS; rho += nparts) {
    const RowAddr a = row_addr<L, M>(c, rowj, 0u, __builtin_amdgcn_readfirstlane(rho));
    tile_energy_row<L, M, 0>(c, a, U);
  }
  return U;
}

// ---------------------------------------------------------------------------
// kernels.  Each works on a set of populations (BatchDev) through a Group that
// assigns workgroups to member populations.
// ---------------------------------------------------------------------------
struct Member {
  uint32_t pop;  // index into B.pops
  uint32_t lb;   // workgroup index within the member
  uint32_t nb;   // workgroups of the member
  uint32_t m;    // member index within the group
};

// The hardware deals the workgroups of a launch round-robin to the 8 XCDs
// (workgroup b to XCD b mod 8), each with its own L2.  xcd_block renumbers
// blocks 0 .. nb-1 so that each XCD takes one contiguous range: XCD x takes
// the x-th range (ranges as equal as possible), so neighbouring tiles, which
// read overlapping old tiles in the gather, share an L2.  A bijection on
// [0, nb); it needs block numbers whose residue mod 8 is the XCD, which holds
// within a population because its sweep blocks start at a multiple of 8.
constexpr uint32_t kXcds = 8;

__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t xcd = b % kXcds, idx = b / kXcds;
  const uint32_t base = nb / kXcds, rem = nb % kXcds;
  return xcd < rem ? xcd * (base + 1) + idx : rem * (base + 1) + (xcd - rem) * base + idx;
}

__device__ __forceinline__ Member member_of_block(const Group& g, uint32_t b) {
  uint32_t lo = 0, hi = g.n;  // start[lo] <= b < start[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (g.start[mid] <= b) lo = mid;
    else hi = mid;
  }
  Member r;
  r.m = __builtin_amdgcn_readfirstlane(lo);
  r.pop = __builtin_amdgcn_readfirstlane(g.pop[r.m]);
  const uint32_t s0 = __builtin_amdgcn_readfirstlane(g.start[r.m]);
  r.lb = b - s0;
  r.nb = __builtin_amdgcn_readfirstlane(g.start[r.m + 1]) - s0;
  return r;
}

__device__ __forceinline__ Member member_of(const Group& g) { return member_of_block(g, blockIdx.x); }

__device__ __forceinline__ uint32_t step_index(const BatchDev& B) {
  return B.steps ? __builtin_amdgcn_readfirstlane(*B.step_ctr) : 0u;
}

// Element b (0 or 1) of a two-entry array of a descriptor, by select: indexing
// the array with a run-time value would make the compiler copy the whole
// descriptor to per-lane scratch memory.
template <typename T>
__device__ __forceinline__ T pick(const T (&a)[2], uint32_t b) {
  return b ? a[1] : a[0];
}

__device__ __forceinline__ PopStep step_of(const BatchDev& B, uint32_t pop) {
  if (!B.steps) return B.single;
  return B.steps[(size_t)step_index(B) * B.n_pops + pop];
}

__device__ __forceinline__ StepRecord* record_of(const BatchDev& B, uint32_t pop) {
  return B.records ? B.records + (size_t)step_index(B) * B.n_pops + pop : nullptr;
}

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
  store_tile<LAYOUT>(lds, pick(P.spins, cur), P.N, tile, 0u, 1u);
  if (valid) {
    pick(P.U, cur)[r] = U;
    pick(P.fam, cur)[r] = r;
  }
}

// Zero the per-step accumulators of each population (one workgroup each).
__global__ __launch_bounds__(256) void k_zero_acc(BatchDev B, Group G) {
  const Member m = member_of(G);
  const DevPop& P = B.pops[m.pop];
  if (P.sc->dead) return;
  // kModelGauss16: the host clears the occupied window once it is known
  if (P.model != kModelGauss16)
    for (uint32_t i = threadIdx.x; i < P.n_levels; i += blockDim.x) P.hist[i] = 0;
  if (threadIdx.x == 0) {
    P.sc->sum_eta2 = 0;
    P.sc->E_lo = 0x7FFFFFFF;
    P.sc->E_hi = (int32_t)0x80000000;
  }
}

// The words of this thread's slots among a workgroup's kHistSlots (slot
// i0 + threadIdx.x + 256 k for a 256-thread workgroup), loaded together: one
// memory round trip rather than one per word.  Slots at or past i1 are not
// read; their entries are left undefined and the caller skips them.
constexpr uint32_t kHistPer = kHistSlots / 256;
__device__ __forceinline__ void slot_words(const uint32_t* U, uint32_t i0, uint32_t i1,
                                           uint32_t u[kHistPer]) {
  const __attribute__((address_space(1))) uint32_t* const Ug =
      (const __attribute__((address_space(1))) uint32_t*)U;
#pragma unroll
  for (uint32_t k = 0; k < kHistPer; ++k) {
    const uint32_t i = i0 + threadIdx.x + 256u * k;
    u[k] = i < i1 ? Ug[i] : 0u;
  }
}

// Energy histogram h_j = #{i < R~ : U_i = j} (the sum of Eq. 2 regrouped by
// integer level), privatised in LDS; each workgroup takes kHistSlots slots.
__global__ __launch_bounds__(256) void k_hist(BatchDev B, Group G, uint32_t post) {
  extern __shared__ uint32_t h[];
  const Member m = member_of(G);
  const DevPop P = B.pops[m.pop];
  const PopStep sp = step_of(B, m.pop);
  const uint32_t* U = pick(P.U, post ? sp.cur ^ 1u : sp.cur);
  // the population's flag and size and the thread's slot words read together
  // (every slot below the capacity is allocated), then the flag checked
  const uint32_t dead = P.sc->dead, R = P.sc->R_tilde;
  const uint32_t i0 = m.lb * kHistSlots, i1 = min(R, i0 + kHistSlots);
  uint32_t u[kHistPer];
  slot_words(U, i0, min(P.capacity, i0 + kHistSlots), u);
  asm volatile("" ::"v"(R));
  if (dead) return;
  for (uint32_t i = threadIdx.x; i < P.n_levels; i += blockDim.x) h[i] = 0;
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < kHistPer; ++k)
    if (i0 + threadIdx.x + 256u * k < i1 && u[k] < P.n_levels) atomicAdd(&h[u[k]], 1u);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < P.n_levels; i += blockDim.x)
    if (h[i]) atomicAdd(&P.hist[i], h[i]);
}

// Position of this thread's element among the flagged elements of the block,
// in thread order (wave ballots + per-wave counts in LDS); *total receives
// the number of flagged elements.  Every thread of the block must call it.
template <int BLOCK>
__device__ uint32_t block_compact_pos(bool flag, uint32_t* wcount, uint32_t* total) {
  constexpr int NW = BLOCK / kWave;
  const uint32_t lane = lane_id(), wid = threadIdx.x / kWave;
  const unsigned long long b = __ballot(flag);
  const uint32_t below = (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
  __syncthreads();  // wcount may still be read from the previous call
  if (lane == 0) wcount[wid] = (uint32_t)__popcll(b);
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t c = wcount[w];
    off += (uint32_t)w < wid ? c : 0u;
    tot += c;
  }
  *total = tot;
  return off + below;
}

// kModelGauss16: lowest and highest E16 of the population.  Each workgroup
// takes kHistSlots slots, reduces them, and adds one atomic min and max.
__global__ __launch_bounds__(256) void k_minmax(BatchDev B, Group G, uint32_t post) {
  __shared__ int32_t smin[256 / kWave], smax[256 / kWave];
  const Member m = member_of(G);
  const DevPop P = B.pops[m.pop];
  if (P.sc->dead) return;
  const PopStep sp = step_of(B, m.pop);
  const uint32_t* U = pick(P.U, post ? sp.cur ^ 1u : sp.cur);
  const uint32_t R = P.sc->R_tilde;
  const uint32_t i0 = m.lb * kHistSlots, i1 = min(R, i0 + kHistSlots);
  if (i0 >= R) return;
  int32_t lo = 0x7FFFFFFF, hi = (int32_t)0x80000000;
  uint32_t u[kHistPer];
  slot_words(U, i0, i1, u);
#pragma unroll
  for (uint32_t k = 0; k < kHistPer; ++k)
    if (i0 + threadIdx.x + 256u * k < i1) {
      lo = min(lo, (int32_t)u[k]);
      hi = max(hi, (int32_t)u[k]);
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = min(lo, __shfl_xor(lo, off, kWave));
    hi = max(hi, __shfl_xor(hi, off, kWave));
  }
  const uint32_t wid = threadIdx.x / kWave;
  if (lane_id() == 0) {
    smin[wid] = lo;
    smax[wid] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256 / kWave; ++w) {
      lo = min(lo, smin[w]);
      hi = max(hi, smax[w]);
    }
    atomicMin(&P.sc->E_lo, lo);
    atomicMax(&P.sc->E_hi, hi);
  }
}

// kModelGauss16: h[E16 - E_lo] over the occupied window of n_win levels
// (global histogram cleared beforehand).  Each workgroup takes kHistSlots
// slots; with LDS (n_win <= kWindowLdsLevels, n_win * 4 bytes of dynamic LDS)
// it counts them in LDS and adds its nonzero bins, else it adds to the global
// bins directly.
__global__ __launch_bounds__(256) void k_hist_window(BatchDev B, Group G, uint32_t n_win,
                                                     uint32_t use_lds) {
  extern __shared__ uint32_t hl[];
  const Member m = member_of(G);
  const DevPop P = B.pops[m.pop];
  if (P.sc->dead) return;
  const PopStep sp = step_of(B, m.pop);
  const uint32_t* U = pick(P.U, sp.cur);
  const uint32_t R = P.sc->R_tilde;
  const int32_t lo = P.sc->E_lo;
  const uint32_t i0 = m.lb * kHistSlots, i1 = min(R, i0 + kHistSlots);
  if (i0 >= R) return;
  if (use_lds) {
    for (uint32_t b = threadIdx.x; b < n_win; b += blockDim.x) hl[b] = 0;
    uint32_t u[kHistPer];
    slot_words(U, i0, i1, u);
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kHistPer; ++k) {
      const int32_t lev = (int32_t)u[k] - lo;
      if (i0 + threadIdx.x + 256u * k < i1 && lev >= 0 && (uint32_t)lev < n_win)
        atomicAdd(&hl[lev], 1u);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < n_win; b += blockDim.x)
      if (hl[b]) atomicAdd(&P.hist[b], hl[b]);
  } else {
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
      const int32_t lev = (int32_t)U[i] - lo;
      if (lev >= 0 && (uint32_t)lev < n_win && (uint32_t)lev < P.n_levels)
        atomicAdd(&P.hist[lev], 1u);
    }
  }
}

// Resampling table on the device (Sec. II, Eqs. 1-2), the same arithmetic as
// the host builder: j_min = lowest occupied level, w_j = erow[j - j_min]
// (erow holds exp(-dbeta * 2d) from the host's exp), S = sum over occupied
// levels, ascending, of h_j w_j, tau_j = R w_j / S, fl_j = floor(tau_j),
// T_j = ceil(frac(tau_j) 2^53).  The culling fraction (Sec. III.C) is summed
// the same way.  Each rounded product or term depends on its level only, so
// the block forms them in parallel, 1024 levels at a time, packs the occupied
// ones in level order into LDS, and one thread adds them in that order: the
// sums round exactly as the host's sequential loops.  S, j_min and R~ are
// recorded; the host finishes ln Q = ln S - ln R~ - dbeta E_min with its log.
constexpr int kTableBlock = 1024;

__global__ __launch_bounds__(kTableBlock) void k_table(BatchDev B, Group G) {
  __shared__ double part[kTableBlock];
  __shared__ uint32_t wcount[kTableBlock / kWave];
  __shared__ double sS, sacc;
  __shared__ int sjmin;
  const Member m = member_of(G);
  const DevPop P = B.pops[m.pop];
  if (P.sc->dead) return;
  const PopStep sp = step_of(B, m.pop);
  const uint32_t* h = P.hist;
  const uint32_t nl = P.n_levels;
  const double R = (double)P.R;
  if (threadIdx.x == 0) {
    sjmin = 0x7FFFFFFF;
    sS = 0.0;
    sacc = 0.0;
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < nl; j += kTableBlock)
    if (h[j] > 0) atomicMin(&sjmin, (int)j);
  __syncthreads();
  const int jmin = sjmin == 0x7FFFFFFF ? -1 : sjmin;
  if (jmin >= 0) {
    // S = sum_j h_j w_j, ascending over occupied levels
    for (uint32_t base = (uint32_t)jmin; base < nl; base += kTableBlock) {
      const uint32_t j = base + threadIdx.x;
      const uint32_t hj = j < nl ? h[j] : 0u;
      uint32_t n;
      const uint32_t pos = block_compact_pos<kTableBlock>(hj > 0, wcount, &n);
      if (hj > 0) part[pos] = __dmul_rn((double)hj, sp.erow[j - (uint32_t)jmin]);
      __syncthreads();
      if (threadIdx.x == 0) {
        double S = sS;
        for (uint32_t i = 0; i < n; ++i) S = __dadd_rn(S, part[i]);
        sS = S;
      }
    }
    __syncthreads();
    const double S = sS;
    // eps R = sum over occupied levels with tau_j < 1 of h_j (1 - tau_j), ascending
    for (uint32_t base = (uint32_t)jmin; base < nl; base += kTableBlock) {
      const uint32_t j = base + threadIdx.x;
      const uint32_t hj = j < nl ? h[j] : 0u;
      double term = 0.0;
      bool take = false;
      if (hj > 0) {
        const double tau = __ddiv_rn(__dmul_rn(R, sp.erow[j - (uint32_t)jmin]), S);
        take = tau < 1.0;
        term = __dmul_rn((double)hj, __dsub_rn(1.0, tau));
      }
      uint32_t n;
      const uint32_t pos = block_compact_pos<kTableBlock>(take, wcount, &n);
      if (take) part[pos] = term;
      __syncthreads();
      if (threadIdx.x == 0) {
        double acc = sacc;
        for (uint32_t i = 0; i < n; ++i) acc = __dadd_rn(acc, part[i]);
        sacc = acc;
      }
    }
  }
  __syncthreads();
  const double S = sS;
  if (threadIdx.x == 0) {
    StepRecord* rec = record_of(B, m.pop);
    if (rec) {
      rec->S = S;
      rec->eps = jmin >= 0 ? __ddiv_rn(sacc, R) : 0.0;
      rec->jmin = jmin;
      rec->R_old = P.sc->R_tilde;
      rec->status = 0;
    }
  }
  if (jmin < 0) return;
  for (uint32_t j = threadIdx.x; j < nl; j += kTableBlock) {
    if ((int)j < jmin) {
      P.table[j].fl = 0;
      P.table[j].T = 0;
      continue;
    }
    const double w = sp.erow[j - (uint32_t)jmin];
    const double tau = __ddiv_rn(__dmul_rn(R, w), S);
    const double f = floor(tau);
    const double fr = __dsub_rn(tau, f);
    P.table[j].fl = (uint32_t)f;
    P.table[j].T = (unsigned long long)ceil(ldexp(fr, 53));
  }
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
// u53 = (w0 << 21) | (w1 >> 11) from Philox(seed; i, step, 0, RES).  The
// table comes from the workspace, or (INLINE) from the kernel's argument,
// which holds the occupied levels j0 .. j0 + n - 1.
template <bool INLINE>
__device__ __forceinline__ TableEntry table_entry(const DevPop& P, const InlineTable* t,
                                                  uint32_t lev) {
  if constexpr (INLINE) {
    const uint32_t k = lev - t->j0;
    return t->e[k < t->n ? k : t->n - 1];
  } else {
    return P.table[min(lev, P.n_levels - 1)];
  }
}

template <bool INLINE>
__device__ __forceinline__ void counts_body(BatchDev B, Group G, const InlineTable* t) {
  __shared__ uint32_t scratch[kBlockCounts / kWave];
  const Member m = member_of(G);
  const DevPop P = B.pops[m.pop];
  const PopStep sp = step_of(B, m.pop);
  const uint32_t* U = pick(P.U, sp.cur);
  const uint32_t i = m.lb * kBlockCounts + threadIdx.x;
  // the population's flag and size and this slot's word read together (every
  // slot below the capacity is allocated), then the flag checked; the asm
  // keeps the compiler from moving the loads below the check
  const uint32_t dead = P.sc->dead, R = P.sc->R_tilde, E_lo = (uint32_t)P.sc->E_lo;
  const uint32_t word = i < P.capacity ? U[i] : 0u;
  asm volatile("" ::"v"(R), "v"(E_lo), "v"(word));
  if (dead) return;
  uint32_t n = 0, culled = 0;
  if (i < R) {
    // energy level of the replica: U (kModelPm) or E16 - E_lo (kModelGauss16)
    const uint32_t lev = P.model == kModelGauss16 ? word - E_lo : word;
    const Words4 w = philox10(i, sp.step, 0u, kTagRes, (uint32_t)P.seed, (uint32_t)(P.seed >> 32));
    const unsigned long long u53 = ((unsigned long long)w.w[0] << 21) | (w.w[1] >> 11);
    const TableEntry te = table_entry<INLINE>(P, t, lev);
    n = te.fl + (u53 < te.T ? 1u : 0u);
    P.counts[i] = n;
    culled = n == 0;
  }
  const uint32_t s = block_sum<kBlockCounts, uint32_t>(n, scratch);
  const uint32_t c = block_sum<kBlockCounts, uint32_t>(culled, scratch);
  if (threadIdx.x == 0) {
    P.block_sums[m.lb] = s;
    P.block_culled[m.lb] = c;
  }
}

__global__ __launch_bounds__(kBlockCounts) void k_counts(BatchDev B, Group G) {
  counts_body<false>(B, G, nullptr);
}

__global__ __launch_bounds__(kBlockCounts) void k_counts_inline(BatchDev B, Group G,
                                                                InlineTable t) {
  counts_body<true>(B, G, &t);
}

// Exclusive scan of the per-block sums (one workgroup per population), the
// new population size R~' = sum n_i, and the capacity check.
__global__ __launch_bounds__(1024) void k_scan(BatchDev B, Group G) {
  __shared__ uint32_t scratch[1024 / kWave];
  __shared__ unsigned long long cull_scratch[1024 / kWave];
  const Member m = member_of(G);
  const DevPop P = B.pops[m.pop];
  if (P.sc->dead) return;
  const PopStep sp = step_of(B, m.pop);
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
  if (sp.flags & kStepHist) {  // for the histogram and family sums after the sweep
    for (uint32_t j = threadIdx.x; j < P.n_levels; j += 1024) P.hist[j] = 0;
    if (threadIdx.x == 0) P.sc->sum_eta2 = 0;
  }
  if (threadIdx.x == 0) {
    const bool over = total > P.cap_limit;
    P.sc->R_next = total;
    P.sc->err = over ? 1u : 0u;
    P.sc->n_culled = (uint32_t)ctot;
    StepRecord* rec = record_of(B, m.pop);
    if (rec) {
      rec->n_culled = (uint32_t)ctot;
      rec->status = over ? 1u : 0u;
    }
    if (over && (sp.flags & kStepSticky)) P.sc->dead = 1u;
  }
}

// Offsets and the new-slot -> old-slot map of the order-preserving copy:
// the n_i copies of old slot i take new slots offset_i .. offset_i + n_i - 1.
// The block's new slots are written by all its threads together, slot j of
// the block's range by thread j mod kBlockCounts: its source is the last old
// slot t of the block whose exclusive offset is <= j (that slot has n_t > 0),
// found by bisection over the offsets in LDS.  A step that gives one replica
// many copies therefore costs no more than one that spreads them.
__global__ __launch_bounds__(kBlockCounts) void k_scatter(BatchDev B, Group G) {
  __shared__ uint32_t scratch[kBlockCounts / kWave];
  __shared__ uint32_t excl_s[kBlockCounts];
  const Member m = member_of(G);
  const DevPop P = B.pops[m.pop];
  if (P.sc->dead || P.sc->err) return;
  const uint32_t R = P.sc->R_tilde;
  const uint32_t i = m.lb * kBlockCounts + threadIdx.x;
  const uint32_t n = i < R ? P.counts[i] : 0u;
  uint32_t total;
  const uint32_t excl = block_exclusive_scan<kBlockCounts>(n, &total, scratch);
  const uint32_t base = P.block_offsets[m.lb];
  if (i < R) P.offsets[i] = base + excl;
  excl_s[threadIdx.x] = excl;
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < total; j += kBlockCounts) {
    uint32_t lo = 0, hi = kBlockCounts;  // excl_s[lo] <= j < excl_s[hi] (excl_s[kBlockCounts] = total)
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (excl_s[mid] <= j)
        lo = mid;
      else
        hi = mid;
    }
    P.src[base + j] = m.lb * kBlockCounts + lo;
  }
}

// The scan and the copy map of one population in one launch (calls on single
// instances): workgroup b starts its new slots at the sum of the block sums
// before it, then maps them as k_scatter does.  The last workgroup, whose
// range ends at the new size R~', records it with the capacity check and the
// culled count, and (kStepHist) clears the histogram and the family sum, as
// k_scan does.  A workgroup whose range would pass the capacity writes
// nothing; the overflow flag then keeps the sweep from applying the step.
__global__ __launch_bounds__(kBlockCounts) void k_scan_scatter(BatchDev B, Group G) {
  __shared__ uint32_t scratch[kBlockCounts / kWave];
  __shared__ uint32_t excl_s[kBlockCounts];
  __shared__ uint32_t s_base;
  const Member m = member_of(G);
  const DevPop P = B.pops[m.pop];
  const PopStep sp = step_of(B, m.pop);
  // the population's flag and size and this slot's count read together
  // (every slot below the capacity is allocated), then the flag checked
  const uint32_t i = m.lb * kBlockCounts + threadIdx.x;
  const uint32_t dead = P.sc->dead, R = P.sc->R_tilde;
  const uint32_t cnt = i < P.capacity ? P.counts[i] : 0u;
  asm volatile("" ::"v"(R), "v"(cnt));
  if (dead) return;
  const uint32_t n = i < R ? cnt : 0u;
  // the block sums before this workgroup, four per 16-byte load (the array
  // starts 256-byte aligned), the last lb mod 4 one by one; the unrolled
  // loop keeps several loads of a thread in flight
  uint32_t before = 0;
  const uint32_t q = m.lb / 4;
  const uint4* bs4 = reinterpret_cast<const uint4*>(P.block_sums);
#pragma unroll 4
  for (uint32_t b = threadIdx.x; b < q; b += kBlockCounts) {
    const uint4 v = bs4[b];
    before += v.x + v.y + v.z + v.w;
  }
  for (uint32_t b = 4 * q + threadIdx.x; b < m.lb; b += kBlockCounts) before += P.block_sums[b];
  before = block_sum<kBlockCounts, uint32_t>(before, scratch);
  if (threadIdx.x == 0) s_base = before;
  __syncthreads();
  const uint32_t base = s_base;
  uint32_t total;
  const uint32_t excl = block_exclusive_scan<kBlockCounts>(n, &total, scratch);
  const bool fits = (unsigned long long)base + total <= P.cap_limit;
  if (fits && i < R) P.offsets[i] = base + excl;
  excl_s[threadIdx.x] = excl;
  __syncthreads();
  if (fits) {
    for (uint32_t j = threadIdx.x; j < total; j += kBlockCounts) {
      uint32_t lo = 0, hi = kBlockCounts;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (excl_s[mid] <= j)
          lo = mid;
        else
          hi = mid;
      }
      P.src[base + j] = m.lb * kBlockCounts + lo;
    }
  }
  if (m.lb + 1 != m.nb) return;
  uint32_t cull = 0;
#pragma unroll 8
  for (uint32_t b = threadIdx.x; b < m.nb; b += kBlockCounts) cull += P.block_culled[b];
  cull = block_sum<kBlockCounts, uint32_t>(cull, scratch);
  if (sp.flags & kStepHist) {
    for (uint32_t j = threadIdx.x; j < P.n_levels; j += kBlockCounts) P.hist[j] = 0;
  }
  if (threadIdx.x == 0) {
    const uint32_t all = base + total;
    P.sc->R_next = all;
    P.sc->err = all > P.cap_limit ? 1u : 0u;
    P.sc->n_culled = cull;
    if (sp.flags & kStepHist) P.sc->sum_eta2 = 0;
  }
}

// Gather (optional) + n_sweeps checkerboard Metropolis sweeps + energy for
// one 64-replica tile per workgroup.  Reads buffer cur, writes buffer cur ^ 1.
// SPLIT wavefronts share the tile's LDS image: each takes every SPLIT-th
// group of eight sites in the gather and the store, and every SPLIT-th block
// of four rows in each colour pass (same-colour sites are independent), with
// a workgroup barrier between colours.  Every lane still owns one replica, and
// every draw is addressed by (slot, sweep, site group), so the split changes
// nothing in the results.  Sharing a tile among waves keeps SPLIT times more
// waves in flight per tile than one wave per tile would, and shortens the walk
// of each tile by the same factor.
//
// Register budget: as many waves per SIMD as fit without spilling to scratch
// memory (+-J: eight up to L = 10, seven at L = 12, six above; quantised
// Gaussian couplings, whose update holds six coupling values: seven up to
// L = 8, six at 10, five at 12 and 14, four at 16).
template <int L, int M>
constexpr int sweep_min_waves_per_eu() {
  if constexpr (M == (int)kModelGauss16) return L <= 8 ? 7 : L == 10 ? 6 : L <= 14 ? 5 : 4;
  if constexpr (M == (int)kModelReal) return L <= 8 ? 7 : L == 10 ? 6 : L <= 14 ? 5 : 4;
  return L <= 10 ? 8 : L == 12 ? 7 : 6;
}

template <int LAYOUT, int L, int SPLIT, int M>
__global__ __launch_bounds__(64 * SPLIT)
__attribute__((amdgpu_waves_per_eu(sweep_min_waves_per_eu<L, M>()))) void k_sweep(BatchDev B,
                                                                                Group G) {
  constexpr uint32_t N = L * L * L;
  __shared__ unsigned long long thr_of_nu[8];  // first LDS object: address 0 (see chunk_sites)
  extern __shared__ uint32_t lds_all[];
  const Member m = member_of(G);
  const DevPop P = B.pops[m.pop];
  if (P.sc->dead) return;
  const PopStep sp = step_of(B, m.pop);
  const uint32_t lane = lane_id();
  // this wave's share of the tile (uniform: a scalar register)
  const uint32_t part = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  // a copy step the scan found over capacity is not applied: nothing runs
  if (sp.gather && P.sc->err != 0u) return;
  if (sp.gather && m.lb == 0 && threadIdx.x == 0) P.sc->R_tilde = P.sc->R_next;
  // uniform: held in a scalar register
  const uint32_t Rs =
      __builtin_amdgcn_readfirstlane(sp.gather ? P.sc->R_next : P.sc->R_tilde);
  // the tiles that hold replicas are spread over the XCDs in contiguous
  // ranges; blocks past them keep their number and leave
  const uint32_t active = (Rs + 63) / 64;
  const uint32_t tile =
      __builtin_amdgcn_readfirstlane(m.lb < active ? xcd_block(m.lb, active) : m.lb);
  // whole workgroups leave together (the passes below use workgroup barriers)
  if (tile * 64 >= Rs) return;
  // Phase 2 of the +-J pass indexes the threshold table by byte address 8 nu:
  // it must sit at LDS address 0; phase 1 of the colour passes reads the tile
  // image at the absolute addresses of its site table, so the image must start
  // at kTileLdsBase; the Gaussian pass reads the dE16 table at the address
  // that follows from both.  If the toolchain ever places them elsewhere, report a
  // configuration error instead of computing with wrong addresses.
  if ((uint32_t)(uintptr_t)thr_of_nu != 0u || (uint32_t)(uintptr_t)lds_all != kTileLdsBase) {
    if (threadIdx.x == 0) {
      P.sc->err = 2u;
      P.sc->dead = 1u;
    }
    return;
  }
  if (threadIdx.x < 8)
    thr_of_nu[threadIdx.x] = threadIdx.x == 0   ? sp.thr[2]
                             : threadIdx.x == 1 ? sp.thr[1]
                             : threadIdx.x == 2 ? sp.thr[0]
                                                : (1ull << 32);
  uint32_t* const lds = lds_all;
  // kModelGauss16: the dE16 threshold table, after the tile image and the
  // waves' plane areas (visible after the gather's barrier)
  unsigned long long* const gtab =
      reinterpret_cast<unsigned long long*>(lds_all + 2 * N + kPlaneAreaBytes / 4 * SPLIT);
  if constexpr (M == (int)kModelGauss16) {
    for (uint32_t i = threadIdx.x; i <= (uint32_t)kGaussDEMax; i += 64 * SPLIT) gtab[i] = P.gthr[i];
  }
  const uint32_t j = tile * 64 + lane;
  const bool valid = j < Rs;
  const uint32_t src = valid ? (sp.gather ? P.src[j] : j) : 0u;
  load_tile_gather<LAYOUT, N>(lds, pick(P.spins, sp.cur), src, valid, part, SPLIT);
  TileCtx c;
  c.lds = lds;
  c.thr_of_nu = thr_of_nu;
  c.hoff = 4u * (lane >> 5);
  c.pos = lane & 31u;
  c.ph.init(j, (uint32_t)P.seed, (uint32_t)(P.seed >> 32));
  // A draw matters only for a class whose threshold is neither 0 nor 2^32.
  // (kModelGauss16: the host passes the largest and the smallest threshold of
  // a positive move, the table's dE16 = 2 and last entries, in thr[0] and
  // thr[1], and 0 in thr[2]; the table is non-increasing, so a draw matters
  // unless both are 0 or both are 2^32.)
  c.writers = 0x0000000100000001ull;
  c.hshift = 8u * c.hoff;
  c.any_draw = (sp.thr[0] != 0 && sp.thr[0] < (1ull << 32)) ||
               (sp.thr[1] != 0 && sp.thr[1] < (1ull << 32)) ||
               (sp.thr[2] != 0 && sp.thr[2] < (1ull << 32));
  c.rowk = P.rowk;
  c.rowk_stride = P.rowk_stride;
  c.gaddr = P.gaddr;
  c.rthr = P.rthr;
  c.rthr32 = P.rthr32;
  c.rhe = P.rhe;
  const unsigned long long* rowj = P.rowj;
  typename AccOf<M>::type U;
  if (sp.n_sweeps == 0) {
    U = tile_energy_rows<L, M>(c, rowj, part, SPLIT);
  } else {
    // this wave's plane area (phase 1 of the colour passes), after the tile
    // image, and the lane's byte address in it for each rotation
    char* const planes = reinterpret_cast<char*>(lds_all + 2 * N) + kPlaneAreaBytes * part;
    PlaneReads pr;
    {
      const uint32_t pb = plane_byte(lane);
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k)
        pr.at[k] = reinterpret_cast<const uint8_t*>(planes) + 16u * (((pb >> 4) + k) & 3u) +
                   (pb & 15u);
    }
    if constexpr (M != (int)kModelPm) {
      for (uint32_t s = 0; s + 1 < sp.n_sweeps; ++s) {
        c.t = sp.t0 + s;
        sweep_colour_patterns<L, SPLIT, M, false>(c, P.psites, 0u, part, planes, pr, lane);
        sweep_colour_patterns<L, SPLIT, M, false>(c, P.psites, 1u, part, planes, pr, lane);
      }
      c.t = sp.t0 + sp.n_sweeps - 1;
      sweep_colour_patterns<L, SPLIT, M, false>(c, P.psites, 0u, part, planes, pr, lane);
      U = sweep_colour_patterns<L, SPLIT, M, true>(c, P.psites, 1u, part, planes, pr, lane);
    } else {
      // every move that raises the energy has a threshold below 2^32 (beta
      // not 0 in double precision): the passes take the 32-bit form, but for
      // the last colour-1 pass, which also sums the energy
      const bool fast = sp.thr[0] < (1ull << 32);
      for (uint32_t s = 0; s < sp.n_sweeps; ++s) {
        c.t = sp.t0 + s;
        for (uint32_t colour = 0; colour < 2; ++colour) {
          if (s + 1 == sp.n_sweeps && colour == 1)
            U = sweep_colour_planes<L, SPLIT, false, true>(c, P.psites, 1u, part, planes, pr,
                                                           lane);
          else if (fast)
            sweep_colour_planes<L, SPLIT, true, false>(c, P.psites, colour, part, planes, pr,
                                                       lane);
          else
            sweep_colour_planes<L, SPLIT, false, false>(c, P.psites, colour, part, planes, pr,
                                                        lane);
        }
      }
    }
  }
  // Epilogue.  The lane number, the slot, its source and the descriptor
  // fields are formed or read again here rather than held in registers
  // through the sweeps (held, some are spilled to scratch memory); the asm
  // statements keep the compiler from reusing the first values.
  uint32_t lane2, pop2 = m.pop;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(lane2));
  asm volatile("" : "+s"(pop2));
  // per-replica sum of the waves' shares (after the tile image, in LDS: the
  // +-J plane areas, free once every wave has passed the barrier below)
  using Acc = typename AccOf<M>::type;
  Acc* const ured = reinterpret_cast<Acc*>(lds_all + 2 * N);
  __syncthreads();
  ured[part * 64 + lane2] = U;
  __syncthreads();
  U = 0;
#pragma unroll
  for (uint32_t w = 0; w < (uint32_t)SPLIT; ++w) U += ured[w * 64 + lane2];
  const DevPop P2 = B.pops[pop2];
  const PopStep sp2 = step_of(B, pop2);
  const uint32_t cur2 = sp2.cur, nxt2 = cur2 ^ 1u;
  store_tile<LAYOUT>(lds, pick(P2.spins, nxt2), N, tile, part, SPLIT);
  const uint32_t j2 = tile * 64 + lane2;
  if (j2 < Rs && part == 0) {
    const uint32_t src2 = sp2.gather ? P2.src[j2] : j2;
    if constexpr (M == (int)kModelReal)
      reinterpret_cast<long long*>(pick(P2.U, nxt2))[j2] = U;
    else
      pick(P2.U, nxt2)[j2] = U;
    pick(P2.fam, nxt2)[j2] = pick(P2.fam, cur2)[src2];
  }
}

// The energy word recomputed from the stored spins of buffer cur (after an
// import; for kModelGauss16 also after the initial spins are drawn), or, with
// CHECK, compared with the stored word (the debug energy check).
template <int LAYOUT, int L, int M, bool CHECK>
__global__ __launch_bounds__(64) void k_energy(BatchDev B, Group G) {
  constexpr uint32_t N = L * L * L;
  extern __shared__ uint32_t lds[];
  const Member m = member_of(G);
  const DevPop P = B.pops[m.pop];
  const PopStep sp = step_of(B, m.pop);
  const uint32_t R = P.sc->R_tilde;
  const uint32_t tile = m.lb;
  if (tile * 64 >= R) return;
  const uint32_t lane = lane_id();
  const uint32_t j = tile * 64 + lane;
  const bool valid = j < R;
  load_tile_gather<LAYOUT, N>(lds, pick(P.spins, sp.cur), valid ? j : 0u, valid, 0u, 1u);
  TileCtx c;
  c.lds = lds;
  c.hoff = 4u * (lane >> 5);
  c.pos = lane & 31u;
  c.rowk = P.rowk;
  c.rowk_stride = P.rowk_stride;
  c.rhe = P.rhe;
  const typename AccOf<M>::type U = tile_energy_rows<L, M>(c, P.rowj, 0u, 1u);
  using Word = typename AccOf<M>::type;
  Word* const words = reinterpret_cast<Word*>(pick(P.U, sp.cur));
  if (CHECK) {
    const bool bad = valid && words[j] != U;
    const unsigned long long m = __ballot(bad);
    if (lane == 0 && m) atomicAdd(&P.sc->check_bad, (uint32_t)__popcll(m));
  } else if (valid) {
    words[j] = U;
  }
}

// Sum over families of eta^2 (Sec. III.A) from the family labels, which stay
// sorted under the order-preserving copy: each run of equal labels is one
// family.  Its first slot i finds the run's end by galloping (probes at i + 1,
// i + 2, i + 4, ... until one leaves the run) and then bisecting the last gap,
// so a family of eta replicas costs about 2 log2(eta) dependent loads.  Only
// the first kFamilyBlocks workgroups of a population work (the rest leave at
// once), each over a stride of the slots, so that few atomic adds reach the
// population's counter.
constexpr uint32_t kFamilyBlocks = 512;

__global__ __launch_bounds__(256) void k_family(BatchDev B, Group G, uint32_t post) {
  __shared__ unsigned long long scratch[256 / kWave];
  const Member m = member_of(G);
  if (m.lb >= kFamilyBlocks) return;
  const DevPop P = B.pops[m.pop];
  if (P.sc->dead) return;
  const PopStep sp = step_of(B, m.pop);
  const uint32_t* fam = pick(P.fam, post ? sp.cur ^ 1u : sp.cur);
  const uint64_t R = P.sc->R_tilde;
  unsigned long long sq = 0;
  for (uint64_t i = (uint64_t)m.lb * 256 + threadIdx.x; i < R; i += (uint64_t)kFamilyBlocks * 256) {
    const uint32_t f = fam[i];
    if (i > 0 && fam[i - 1] == f) continue;
    // [i, in) lies in the run; the run ends at or before `out`
    uint64_t in = i + 1, out = in, step = 1;
    while (out < R && fam[out] == f) {
      in = out + 1;
      step <<= 1;
      out = i + step;
    }
    uint64_t lo = in, hi = out < R ? out : R;
    while (lo < hi) {  // first index in [lo, hi) with fam != f, else hi
      const uint64_t mid = lo + (hi - lo) / 2;
      if (fam[mid] == f) lo = mid + 1;
      else hi = mid;
    }
    const unsigned long long eta = lo - i;
    sq += eta * eta;
  }
  const unsigned long long s = block_sum<256, unsigned long long>(sq, scratch);
  if (threadIdx.x == 0 && s) atomicAdd(&P.sc->sum_eta2, s);
}

// Post-step record of a batch step: integer sum of E over the population, the
// lowest energy, the new size and the family sum (one workgroup each).
__global__ __launch_bounds__(256) void k_record(BatchDev B, Group G) {
  __shared__ long long scratch[256 / kWave];
  __shared__ int smin;
  const Member m = member_of(G);
  const DevPop P = B.pops[m.pop];
  StepRecord* rec = record_of(B, m.pop);
  if (!rec) return;
  if (P.sc->err == 2u) {  // the sweep did not run: report it, and nothing else
    if (threadIdx.x == 0) rec->status = 2u;
    return;
  }
  if (P.sc->dead) return;
  if (threadIdx.x == 0) smin = 0x7FFFFFFF;
  __syncthreads();
  long long acc = 0;
  const int N3 = 3 * (int)P.N;
  for (uint32_t j = threadIdx.x; j < P.n_levels; j += blockDim.x) {
    const uint32_t hj = P.hist[j];
    if (hj) {
      acc += (long long)hj * (2 * (long long)j - N3);
      atomicMin(&smin, (int)j);
    }
  }
  const long long s = block_sum<256, long long>(acc, scratch);
  if (threadIdx.x == 0) {
    rec->sumE = s;
    rec->E_min = smin == 0x7FFFFFFF ? 0 : 2 * smin - N3;
    rec->n_at_E_min = smin == 0x7FFFFFFF ? 0u : P.hist[smin];
    rec->R_new = P.sc->R_tilde;
    rec->sum_eta2 = P.sc->sum_eta2;
  }
}

// Spin-overlap histogram (Sec. II.A): slot i of population a against slot i
// of population b; d = differing sites, bin = (128 (N - d) + N) / (2N).
// Member m of the group is pair k = G.pop[m] (populations pair_pops[2k], pair_pops[2k+1]).
// One workgroup per 64-pair tile; its kOverlapWaves waves take every
// kOverlapWaves-th site (more loads in flight than one wave per tile) and
// their counts are added per pair through LDS.
constexpr uint32_t kOverlapWaves = 4;

template <int LAYOUT>
__global__ __launch_bounds__(64 * kOverlapWaves) void k_overlap(BatchDev B, Group G,
                                                const uint32_t* __restrict__ pair_pops,
                                                uint32_t post, uint32_t cur_a1, uint32_t cur_b1) {
  __shared__ uint32_t hb[65];
  __shared__ uint32_t dpart[kOverlapWaves][64];
  const Member m = member_of(G);
  const uint32_t k = m.pop;  // pair index
  const uint32_t ia = __builtin_amdgcn_readfirstlane(pair_pops[2 * k]);
  const uint32_t ib = __builtin_amdgcn_readfirstlane(pair_pops[2 * k + 1]);
  const DevPop A = B.pops[ia];
  const DevPop Bp = B.pops[ib];
  if (A.sc->dead || Bp.sc->dead) return;
  // batch steps carry each population's buffer; a call on two instances passes them
  const uint32_t base_a = B.steps ? step_of(B, ia).cur : cur_a1;
  const uint32_t base_b = B.steps ? step_of(B, ib).cur : cur_b1;
  const uint32_t cur_a = post ? base_a ^ 1u : base_a, cur_b = post ? base_b ^ 1u : base_b;
  unsigned long long* out =
      B.qhist ? B.qhist + ((size_t)step_index(B) * B.n_pairs + k) * 65 : A.ovl_hist;
  const uint32_t tile = m.lb;
  const uint32_t lane = lane_id();
  const uint32_t part = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const uint32_t n = min(A.sc->R_tilde, Bp.sc->R_tilde);
  if (tile * 64 >= n) return;
  for (uint32_t b = threadIdx.x; b < 65; b += 64 * kOverlapWaves) hb[b] = 0;
  const uint32_t i = tile * 64 + lane;
  const uint32_t N = A.N;
  uint32_t d = 0;
  if (LAYOUT == 2) {
    const unsigned long long* a = static_cast<const unsigned long long*>(pick(A.spins, cur_a)) +
                                  (size_t)tile * N;
    const unsigned long long* b = static_cast<const unsigned long long*>(pick(Bp.spins, cur_b)) +
                                  (size_t)tile * N;
#pragma unroll 8
    for (uint32_t cm = part; cm < N; cm += kOverlapWaves)
      d += (uint32_t)((a[cm] ^ b[cm]) >> lane) & 1u;
  } else {
    const int8_t* a = static_cast<const int8_t*>(pick(A.spins, cur_a)) + (size_t)tile * N * 64 + lane;
    const int8_t* b = static_cast<const int8_t*>(pick(Bp.spins, cur_b)) + (size_t)tile * N * 64 + lane;
#pragma unroll 8
    for (uint32_t cm = part; cm < N; cm += kOverlapWaves) d += a[64 * (size_t)cm] != b[64 * (size_t)cm];
  }
  dpart[part][lane] = d;
  __syncthreads();
  if (part == 0) {
    d = 0;
#pragma unroll
    for (uint32_t w = 0; w < kOverlapWaves; ++w) d += dpart[w][lane];
    if (i < n) atomicAdd(&hb[(128u * (N - d) + N) / (2u * N)], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < 65; b += 64 * kOverlapWaves)
    if (hb[b]) atomicAdd(&out[b], (unsigned long long)hb[b]);
}

// Link-overlap histogram (Sec. II.A): slot i of population a against slot i
// of population b, one 64-pair tile per wave.  With x_n = s^a_n s^b_n a bond
// <n,m> contributes x_n x_m, so only the bonds whose ends differ in x count:
// D = their number, q_l = 1 - 2 D / (3N), hist[D] += 1 per pair.  The tile's x
// words go to LDS (colour-major, 64 pairs per site, 8N bytes); each lane then
// reads the half word holding its pair.  For even L every bond joins a
// colour-0 site to a colour-1 site, so the walk over the six bonds of every
// colour-0 site counts each bond once.
//
// The colour-0 sites of row (y, z) sit at x = 2q + P, P = (y + z) & 1; their
// +x and -x neighbours are ranks (q + P) and (q + P - 1) mod L/2 of the
// colour-1 row (y, z), their y and z neighbours rank q of the colour-1 rows
// (y +- 1, z) and (y, z +- 1).  Each bond costs one masked XOR (the lane's
// bit of own ^ neighbour) and one popcount-accumulate.
template <int L, int P>
__device__ __forceinline__ uint32_t link_row(const uint32_t* own, const uint32_t* xr,
                                             const uint32_t* py, const uint32_t* my,
                                             const uint32_t* pz, const uint32_t* mz, uint32_t m,
                                             uint32_t d) {
  constexpr int H = L / 2;
#pragma unroll
  for (int q = 0; q < H; ++q) {
    const uint32_t o = own[2 * q];
    const int qp = (q + P) % H, qm = (q + P + H - 1) % H;
    d += __builtin_popcount((o ^ xr[2 * qp]) & m);
    d += __builtin_popcount((o ^ xr[2 * qm]) & m);
    d += __builtin_popcount((o ^ py[2 * q]) & m);
    d += __builtin_popcount((o ^ my[2 * q]) & m);
    d += __builtin_popcount((o ^ pz[2 * q]) & m);
    d += __builtin_popcount((o ^ mz[2 * q]) & m);
  }
  return d;
}

template <int LAYOUT, int L>
__global__ __launch_bounds__(64) void k_link_overlap(DevPop A, DevPop Bp, uint32_t cur_a,
                                                     uint32_t cur_b,
                                                     uint32_t* __restrict__ part) {
  constexpr uint32_t H = L / 2, N = L * L * L;
  __shared__ uint32_t xs[2 * N];  // site cm: words 2 cm (pairs 0..31), 2 cm + 1 (32..63)
  const uint32_t tile = blockIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t n = min(A.sc->R_tilde, Bp.sc->R_tilde);
  if (tile * 64 >= n) return;
  if (LAYOUT == 2) {
    const unsigned long long* a = static_cast<const unsigned long long*>(pick(A.spins, cur_a)) +
                                  (size_t)tile * N;
    const unsigned long long* b = static_cast<const unsigned long long*>(pick(Bp.spins, cur_b)) +
                                  (size_t)tile * N;
    for (uint32_t cm = lane; cm < N; cm += 64) {
      const unsigned long long x = a[cm] ^ b[cm];
      xs[2 * cm] = (uint32_t)x;
      xs[2 * cm + 1] = (uint32_t)(x >> 32);
    }
  } else {
    const int8_t* a = static_cast<const int8_t*>(pick(A.spins, cur_a)) + (size_t)tile * N * 64 + lane;
    const int8_t* b = static_cast<const int8_t*>(pick(Bp.spins, cur_b)) + (size_t)tile * N * 64 + lane;
#pragma unroll 8
    for (uint32_t cm = 0; cm < N; ++cm) {
      const unsigned long long x = __ballot(a[64 * (size_t)cm] != b[64 * (size_t)cm]);
      if (lane == 0) {
        xs[2 * cm] = (uint32_t)x;
        xs[2 * cm + 1] = (uint32_t)(x >> 32);
      }
    }
  }
  __syncthreads();
  const uint32_t* xh = xs + (lane >> 5);
  const uint32_t m = 1u << (lane & 31u);
  uint32_t d = 0;
  for (uint32_t z = 0; z < (uint32_t)L; ++z) {
    const uint32_t zp = z + 1 == (uint32_t)L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
    for (uint32_t y = 0; y < (uint32_t)L; ++y) {
      const uint32_t yp = y + 1 == (uint32_t)L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
      const uint32_t* own = xh + whole_s(2 * H * (y + L * z));
      const uint32_t* xr = xh + whole_s(2 * (N / 2 + H * (y + L * z)));
      const uint32_t* py = xh + whole_s(2 * (N / 2 + H * (yp + L * z)));
      const uint32_t* my = xh + whole_s(2 * (N / 2 + H * (ym + L * z)));
      const uint32_t* pz = xh + whole_s(2 * (N / 2 + H * (y + L * zp)));
      const uint32_t* mz = xh + whole_s(2 * (N / 2 + H * (y + L * zm)));
      if ((y + z) & 1u)
        d = link_row<L, 1>(own, xr, py, my, pz, mz, m, d);
      else
        d = link_row<L, 0>(own, xr, py, my, pz, mz, m, d);
    }
  }
  // each tile counts into copy tile mod kLinkCopies of the histogram, so that
  // concurrent waves rarely update the same word; k_link_reduce sums the copies
  if (tile * 64 + lane < n) atomicAdd(&part[(tile % kLinkCopies) * (3 * N + 1) + d], 1u);
}

// hist[D] = sum over the kLinkCopies partial histograms (nbins = 3N + 1).
__global__ __launch_bounds__(256) void k_link_reduce(const uint32_t* __restrict__ part,
                                                     uint32_t nbins,
                                                     unsigned long long* __restrict__ hist) {
  const uint32_t b = blockIdx.x * 256 + threadIdx.x;
  if (b >= nbins) return;
  unsigned long long acc = 0;
  for (uint32_t k = 0; k < kLinkCopies; ++k) acc += part[(size_t)k * nbins + b];
  hist[b] = acc;
}

__global__ void k_advance(uint32_t* ctr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ctr += 1u;
}

inline uint32_t tiles_of(uint32_t n) { return (n + 63) / 64; }

// ---------------------------------------------------------------------------
// Diagnostics: the device's ceilings for the sweep's roofline.
// ---------------------------------------------------------------------------
// Sustained issue rate of a 32-bit VALU instruction: eight independent chains
// per lane (no chain waits on its own latency), kProbeValuOpsPerIter
// instructions per iteration, a grid of kProbeThreads lanes that fills every
// SIMD.  FORM 0: v_add_u32 (two register sources; on gfx950 such simple
// operations, XOR and v_bitop3_b32 among them, issue faster than one wave per
// four cycles); FORM 1: v_bfe_u32 (three sources, the rate of the sweep's
// bit-field extracts, three-input adds and 24-bit multiply-adds).
template <int FORM>
__global__ __launch_bounds__(256) void k_probe_valu(uint32_t* out, uint32_t iters) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t v0 = gid, v1 = gid + 1, v2 = gid + 2, v3 = gid + 3;
  uint32_t v4 = gid + 4, v5 = gid + 5, v6 = gid + 6, v7 = gid + 7;
  const uint32_t d = gid | 1u;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < kProbeValuOpsPerIter / 8; ++r) {
      if constexpr (FORM == 0)
        asm volatile(
            "v_add_u32 %0, %0, %8\n\tv_add_u32 %1, %1, %8\n\tv_add_u32 %2, %2, %8\n\t"
            "v_add_u32 %3, %3, %8\n\tv_add_u32 %4, %4, %8\n\tv_add_u32 %5, %5, %8\n\t"
            "v_add_u32 %6, %6, %8\n\tv_add_u32 %7, %7, %8"
            : "+v"(v0), "+v"(v1), "+v"(v2), "+v"(v3), "+v"(v4), "+v"(v5), "+v"(v6), "+v"(v7)
            : "v"(d));
      else
        asm volatile(
            "v_bfe_u32 %0, %0, %8, 9\n\tv_bfe_u32 %1, %1, %8, 9\n\tv_bfe_u32 %2, %2, %8, 9\n\t"
            "v_bfe_u32 %3, %3, %8, 9\n\tv_bfe_u32 %4, %4, %8, 9\n\tv_bfe_u32 %5, %5, %8, 9\n\t"
            "v_bfe_u32 %6, %6, %8, 9\n\tv_bfe_u32 %7, %7, %8, 9"
            : "+v"(v0), "+v"(v1), "+v"(v2), "+v"(v3), "+v"(v4), "+v"(v5), "+v"(v6), "+v"(v7)
            : "v"(d));
    }
  }
  out[gid] = v0 ^ v1 ^ v2 ^ v3 ^ v4 ^ v5 ^ v6 ^ v7;
}

// Metropolis draws alone: the sweep's Philox calls (same counter layout and
// hoisting), one call per group g, four draws each, folded into one word so
// that no call is dead.
__global__ __launch_bounds__(256) void k_probe_philox(uint32_t* out, uint32_t calls) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  MetPhilox ph;
  ph.init(gid, 0x5EED1234u, 0xC0DE5678u);
  const uint32_t t = __builtin_amdgcn_readfirstlane(blockIdx.x);
  uint32_t acc = 0;
  for (uint32_t g = 0; g < calls; ++g) {
    const Words4 w = ph.draw(t, g);
    acc ^= w.w[0] ^ w.w[1] ^ w.w[2] ^ w.w[3];
  }
  out[gid] = acc;
}

// the kernels of the real-coupling model (kModelReal)
#include "pa_real_kernels.inc"

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
  const size_t lds = (size_t)P.N * 8;
  if (P.layout == 2)
    hipLaunchKernelGGL(k_init<2>, dim3(tiles_of(P.R)), dim3(64), lds, stream, P, cur,
                       P.cm_of_site);
  else
    hipLaunchKernelGGL(k_init<1>, dim3(tiles_of(P.R)), dim3(64), lds, stream, P, cur,
                       P.cm_of_site);
  return hipGetLastError();
}

hipError_t launch_zero_acc(const BatchDev& B, const Group& g, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_zero_acc, dim3(g.blocks), dim3(256), 0, stream, B, g);
  return hipGetLastError();
}

hipError_t launch_hist(const BatchDev& B, const Group& g, uint32_t max_levels, bool post,
                       hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_hist, dim3(g.blocks), dim3(256), (size_t)max_levels * 4, stream, B, g,
                     post ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_minmax(const BatchDev& B, const Group& g, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_minmax, dim3(g.blocks), dim3(256), 0, stream, B, g, 0u);
  return hipGetLastError();
}

hipError_t launch_hist_window(const BatchDev& B, const Group& g, uint32_t n_win,
                              hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  const bool lds = n_win <= (uint32_t)kWindowLdsLevels;
  hipLaunchKernelGGL(k_hist_window, dim3(g.blocks), dim3(256), lds ? (size_t)n_win * 4 : 0, stream,
                     B, g, n_win, lds ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_table(const BatchDev& B, const Group& g, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_table, dim3(g.blocks), dim3(kTableBlock), 0, stream, B, g);
  return hipGetLastError();
}

hipError_t launch_counts(const BatchDev& B, const Group& g, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_counts, dim3(g.blocks), dim3(kBlockCounts), 0, stream, B, g);
  return hipGetLastError();
}

hipError_t launch_counts_inline(const BatchDev& B, const Group& g, const InlineTable& t,
                                hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_counts_inline, dim3(g.blocks), dim3(kBlockCounts), 0, stream, B, g, t);
  return hipGetLastError();
}

hipError_t launch_scan(const BatchDev& B, const Group& g, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_scan, dim3(g.blocks), dim3(1024), 0, stream, B, g);
  return hipGetLastError();
}

hipError_t launch_scan_scatter(const BatchDev& B, const Group& g, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_scan_scatter, dim3(g.blocks), dim3(kBlockCounts), 0, stream, B, g);
  return hipGetLastError();
}

hipError_t launch_scatter(const BatchDev& B, const Group& g, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3(g.blocks), dim3(kBlockCounts), 0, stream, B, g);
  return hipGetLastError();
}

template <int LAYOUT, int L>
void launch_sweep_l(const BatchDev& B, const Group& g, uint32_t split, uint32_t model,
                    hipStream_t stream) {
  // after the tile image and the reduction area: the Gaussian threshold table,
  // or the +-J plane areas (one per wave)
  // after the tile image: the reduction area and the Gaussian threshold table,
  // or the +-J plane areas (one per wave; the reduction area lies over them)
  const size_t after = model == kModelGauss16
                           ? (size_t)kPlaneAreaBytes * split + (size_t)(kGaussDEMax + 1) * 8
                           : (size_t)kPlaneAreaBytes * split;
  static_assert(kPlaneAreaBytes >= 8 * 64, "the reduction area lies over the plane areas");
  const size_t lds = (size_t)L * L * L * 8 + after;
  if (model == kModelReal) {
    if (split == 8)
      hipLaunchKernelGGL((k_sweep<LAYOUT, L, 8, kModelReal>), dim3(g.blocks), dim3(64 * 8), lds,
                         stream, B, g);
    else
      hipLaunchKernelGGL((k_sweep<LAYOUT, L, 4, kModelReal>), dim3(g.blocks), dim3(64 * 4), lds,
                         stream, B, g);
  } else if (model == kModelGauss16) {
    if (split == 8)
      hipLaunchKernelGGL((k_sweep<LAYOUT, L, 8, kModelGauss16>), dim3(g.blocks), dim3(64 * 8), lds,
                         stream, B, g);
    else
      hipLaunchKernelGGL((k_sweep<LAYOUT, L, 4, kModelGauss16>), dim3(g.blocks), dim3(64 * 4), lds,
                         stream, B, g);
  } else {
    if (split == 8)
      hipLaunchKernelGGL((k_sweep<LAYOUT, L, 8, kModelPm>), dim3(g.blocks), dim3(64 * 8), lds,
                         stream, B, g);
    else
      hipLaunchKernelGGL((k_sweep<LAYOUT, L, 4, kModelPm>), dim3(g.blocks), dim3(64 * 4), lds,
                         stream, B, g);
  }
}

template <int LAYOUT, int L>
void launch_energy_l(const BatchDev& B, const Group& g, uint32_t model, bool check,
                     hipStream_t stream) {
  const size_t lds = (size_t)L * L * L * 8;
  if (model == kModelReal) {
    if (check)
      hipLaunchKernelGGL((k_energy<LAYOUT, L, kModelReal, true>), dim3(g.blocks), dim3(64), lds,
                         stream, B, g);
    else
      hipLaunchKernelGGL((k_energy<LAYOUT, L, kModelReal, false>), dim3(g.blocks), dim3(64), lds,
                         stream, B, g);
  } else if (model == kModelGauss16) {
    if (check)
      hipLaunchKernelGGL((k_energy<LAYOUT, L, kModelGauss16, true>), dim3(g.blocks), dim3(64), lds,
                         stream, B, g);
    else
      hipLaunchKernelGGL((k_energy<LAYOUT, L, kModelGauss16, false>), dim3(g.blocks), dim3(64),
                         lds, stream, B, g);
  } else {
    if (check)
      hipLaunchKernelGGL((k_energy<LAYOUT, L, kModelPm, true>), dim3(g.blocks), dim3(64), lds,
                         stream, B, g);
    else
      hipLaunchKernelGGL((k_energy<LAYOUT, L, kModelPm, false>), dim3(g.blocks), dim3(64), lds,
                         stream, B, g);
  }
}

#define PA_L_SWITCH(FN, LAYOUT)      \
  switch (L) {                       \
    case 4: FN<LAYOUT, 4>(B, g, model, check, stream); break;   \
    case 6: FN<LAYOUT, 6>(B, g, model, check, stream); break;   \
    case 8: FN<LAYOUT, 8>(B, g, model, check, stream); break;   \
    case 10: FN<LAYOUT, 10>(B, g, model, check, stream); break; \
    case 12: FN<LAYOUT, 12>(B, g, model, check, stream); break; \
    case 14: FN<LAYOUT, 14>(B, g, model, check, stream); break; \
    case 16: FN<LAYOUT, 16>(B, g, model, check, stream); break; \
    default: return hipErrorInvalidValue;         \
  }

#define PA_L_SWITCH_S(FN, LAYOUT)                        \
  switch (L) {                                           \
    case 4: FN<LAYOUT, 4>(B, g, split, model, stream); break;   \
    case 6: FN<LAYOUT, 6>(B, g, split, model, stream); break;   \
    case 8: FN<LAYOUT, 8>(B, g, split, model, stream); break;   \
    case 10: FN<LAYOUT, 10>(B, g, split, model, stream); break; \
    case 12: FN<LAYOUT, 12>(B, g, split, model, stream); break; \
    case 14: FN<LAYOUT, 14>(B, g, split, model, stream); break; \
    case 16: FN<LAYOUT, 16>(B, g, split, model, stream); break; \
    default: return hipErrorInvalidValue;                \
  }

hipError_t launch_sweep(const BatchDev& B, const Group& g, uint32_t layout, uint32_t L,
                        uint32_t split, uint32_t model, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  if (split != 4 && split != 8) return hipErrorInvalidValue;
  if (layout == 2) {
    PA_L_SWITCH_S(launch_sweep_l, 2)
  } else {
    PA_L_SWITCH_S(launch_sweep_l, 1)
  }
  return hipGetLastError();
}

hipError_t launch_energy(const BatchDev& B, const Group& g, uint32_t layout, uint32_t L,
                         uint32_t model, bool check, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  if (layout == 2) {
    PA_L_SWITCH(launch_energy_l, 2)
  } else {
    PA_L_SWITCH(launch_energy_l, 1)
  }
  return hipGetLastError();
}
#undef PA_L_SWITCH
#undef PA_L_SWITCH_S

hipError_t launch_family(const BatchDev& B, const Group& g, bool post, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_family, dim3(g.blocks), dim3(256), 0, stream, B, g, post ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_record(const BatchDev& B, const Group& g, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_record, dim3(g.blocks), dim3(256), 0, stream, B, g);
  return hipGetLastError();
}

hipError_t launch_overlap(const BatchDev& B, const Group& g, const uint32_t* pair_pops,
                          uint32_t layout, bool post, uint32_t cur_a, uint32_t cur_b,
                          hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  if (layout == 2)
    hipLaunchKernelGGL(k_overlap<2>, dim3(g.blocks), dim3(64 * kOverlapWaves), 0, stream, B, g, pair_pops,
                       post ? 1u : 0u, cur_a, cur_b);
  else
    hipLaunchKernelGGL(k_overlap<1>, dim3(g.blocks), dim3(64 * kOverlapWaves), 0, stream, B, g, pair_pops,
                       post ? 1u : 0u, cur_a, cur_b);
  return hipGetLastError();
}

template <int LAYOUT>
static hipError_t launch_link_overlap_l(const DevPop& a, const DevPop& b, uint32_t cur_a,
                                        uint32_t cur_b, uint32_t* part, uint32_t tiles,
                                        hipStream_t stream) {
  switch (a.L) {
#define PA_LINK_CASE(LL)                                                                       \
  case LL:                                                                                     \
    hipLaunchKernelGGL((k_link_overlap<LAYOUT, LL>), dim3(tiles), dim3(64), 0, stream, a, b,   \
                       cur_a, cur_b, part);                                                    \
    break;
    PA_LINK_CASE(4) PA_LINK_CASE(6) PA_LINK_CASE(8) PA_LINK_CASE(10) PA_LINK_CASE(12)
    PA_LINK_CASE(14) PA_LINK_CASE(16)
#undef PA_LINK_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_link_overlap(const DevPop& a, const DevPop& b, uint32_t cur_a, uint32_t cur_b,
                               uint32_t* part, unsigned long long* hist, hipStream_t stream) {
  if (a.L != b.L || a.layout != b.layout) return hipErrorInvalidValue;
  const uint32_t tiles = min(a.capacity, b.capacity) / 64;
  const uint32_t nbins = 3 * a.N + 1;
  hipError_t e = hipSuccess;
  if (tiles) {
    e = a.layout == 2 ? launch_link_overlap_l<2>(a, b, cur_a, cur_b, part, tiles, stream)
                      : launch_link_overlap_l<1>(a, b, cur_a, cur_b, part, tiles, stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_link_reduce, dim3((nbins + 255) / 256), dim3(256), 0, stream, part, nbins,
                     hist);
  return hipGetLastError();
}

hipError_t launch_advance(uint32_t* step_ctr, hipStream_t stream) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, stream, step_ctr);
  return hipGetLastError();
}

hipError_t launch_real_thresholds(const DevPop& P, double beta, hipStream_t stream) {
  const uint32_t n = P.N * kRealPatterns;
  hipLaunchKernelGGL(k_rthr, dim3((n + 255) / 256), dim3(256), 0, stream, P, beta);
  return hipGetLastError();
}

hipError_t launch_real_stats(const BatchDev& B, const Group& g, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_rstats, dim3(g.blocks), dim3(kBlockCounts), 0, stream, B, g);
  return hipGetLastError();
}

hipError_t launch_real_sum(const BatchDev& B, const Group& g, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_rsum, dim3(g.blocks), dim3(kBlockCounts), 0, stream, B, g);
  return hipGetLastError();
}

hipError_t launch_real_bisect_init(const DevPop& P, double rem, double target,
                                   hipStream_t stream) {
  hipLaunchKernelGGL(k_rbisect_init, dim3(1), dim3(64), 0, stream, P, rem, target);
  return hipGetLastError();
}

hipError_t launch_real_bisect_eval(const RevalArgs& a, uint32_t blocks, hipStream_t stream) {
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(k_reval, dim3(blocks), dim3(kBlockCounts), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_real_counts(const BatchDev& B, const Group& g, hipStream_t stream) {
  if (!g.blocks) return hipSuccess;
  hipLaunchKernelGGL(k_rcounts, dim3(g.blocks), dim3(kBlockCounts), 0, stream, B, g);
  return hipGetLastError();
}

hipError_t launch_probe_valu(uint32_t* out, uint32_t iters, uint32_t form, hipStream_t stream) {
  if (form == 0)
    hipLaunchKernelGGL(k_probe_valu<0>, dim3(kProbeThreads / 256), dim3(256), 0, stream, out, iters);
  else
    hipLaunchKernelGGL(k_probe_valu<1>, dim3(kProbeThreads / 256), dim3(256), 0, stream, out, iters);
  return hipGetLastError();
}

hipError_t launch_probe_philox(uint32_t* out, uint32_t calls, hipStream_t stream) {
  hipLaunchKernelGGL(k_probe_philox, dim3(kProbeThreads / 256), dim3(256), 0, stream, out, calls);
  return hipGetLastError();
}

}  // namespace pa
