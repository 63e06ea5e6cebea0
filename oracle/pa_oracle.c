/*
 * pa_oracle.c -- plain CPU oracle for population annealing (PA) on the
 * 3D Edwards-Anderson spin glass, with +-J couplings, with Gaussian
 * couplings rounded to multiples of 1/16, and with real Gaussian couplings
 * (FP64 on the grid 2^-32, per-replica weights and fixed-point sums).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant generator with the HIP path; the two meet only
 * through the arithmetic contract written out below.
 *
 * Paper: C. Amey and J. Machta, "Analysis and Optimization of Population
 * Annealing", arXiv:1711.02146 (Sec. II: the algorithm; Sec. II.A: model and
 * observables; Sec. III: rho_t, culling fraction).
 *
 * Everything here is the most direct reading of the paper's steps, kept slow
 * and obvious: spins are int8 +-1 stored [replica][site]; sites are visited
 * in lexicographic order; every random word is drawn with its own Philox call.
 * Built with -ffp-contract=off so every FP64 line rounds as written, left to
 * right.  OpenMP only splits independent replicas; results do not depend on
 * the thread count because every draw is addressed by a counter.
 *
 * Readings where the paper is silent (the coupling distribution, the MCMC
 * variant and its order, the random-number contract, the reference-energy
 * shift, the copy-count tie rule, the constant-culling bisection) are
 * stated at the function that takes them.
 *
 * Parity unpinned: the overlap histogram's bin convention (pao_overlap_hist)
 * and the denominator R of rho_t (pao_sum_eta2's use) are conventions the
 * paper does not fix; no independent value checks them, so they are compared
 * between this oracle and the GPU only.  Everything else is pinned by the CPU
 * tests against closed forms, exact enumeration and the paper's relations.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Counter (c0,c1,c2,c3), key (k0,k1).  Each of   */
/* ten rounds multiplies c0 and c2 by the two round multipliers, swaps the   */
/* halves and XORs in the other counter words and the round key; the key is  */
/* bumped by the two Weyl constants between rounds.                          */
/* ------------------------------------------------------------------------ */
#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u
#define PHILOX_WEYL_B 0xBB67AE85u

/* Stream tags: the fourth counter word separates the three uses of the
 * generator so that no two uses can ever share a counter. */
#define TAG_INIT 0x494E4954u /* initial spins */
#define TAG_MET 0x4D455452u  /* Metropolis acceptance draws */
#define TAG_RES 0x52455341u  /* resampling (copy-count) draws */
#define TAG_J 0x434F5550u    /* +-J couplings of a disorder sample */

void pao_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
    uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)pb;
    uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)pa;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += PHILOX_WEYL_A;
    k1 += PHILOX_WEYL_B;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* +-J couplings of one disorder sample (Sec. II.A, couplings +-1 with
 * probability 1/2): bond b takes +1 when the top bit of word b & 3 of the
 * Philox call with counter (b >> 2, 0, 0, TAG_J) under the coupling seed is
 * clear, -1 when it is set. */
void pao_make_couplings_pm(uint64_t coupling_seed, int L, int8_t* J_out) {
  int64_t nb = 3 * (int64_t)L * L * L;
  uint32_t key[2] = {(uint32_t)coupling_seed, (uint32_t)(coupling_seed >> 32)};
  for (int64_t b = 0; b < nb; ++b) {
    uint32_t ctr[4] = {(uint32_t)(b >> 2), 0u, 0u, TAG_J};
    uint32_t w[4];
    pao_philox(ctr, key, w);
    J_out[b] = (w[b & 3] >> 31) ? -1 : 1;
  }
}

/* One 32-bit word of Philox(seed; c0, c1, c2, tag), word index w in 0..3.
 * The 64-bit population seed is the key: low half first. */
static uint32_t draw_word(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                          uint32_t tag, int w) {
  uint32_t ctr[4] = {c0, c1, c2, tag};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  pao_philox(ctr, key, out);
  return out[w];
}

/* ------------------------------------------------------------------------ */
/* Lattice (Sec. II.A): L^3 cubic lattice, periodic boundaries, Ising spins  */
/* s = +-1, H = -sum_<nm> J_nm s_n s_m over nearest-neighbour bonds.          */
/*   site = x + L*(y + L*z);  bond b = d*N + site joins site and site + e_d   */
/*   (d = 0,1,2 for x,y,z), so every bond is listed exactly once.             */
/*   colour(site) = (x+y+z) & 1.                                              */
/*   cm(site): list the colour-0 sites, then the colour-1 sites, each in      */
/*   lexicographic order; cm is the position of the site in that list.  It is */
/*   computed here by counting.                                               */
/* ------------------------------------------------------------------------ */
static int wrap(int a, int L) { return (a % L + L) % L; }

/* Neighbour of `site` one step along direction dir: 0:+x 1:-x 2:+y 3:-y 4:+z 5:-z */
static int neighbour(int site, int dir, int L) {
  int x = site % L, y = (site / L) % L, z = site / (L * L);
  switch (dir) {
    case 0: x = wrap(x + 1, L); break;
    case 1: x = wrap(x - 1, L); break;
    case 2: y = wrap(y + 1, L); break;
    case 3: y = wrap(y - 1, L); break;
    case 4: z = wrap(z + 1, L); break;
    default: z = wrap(z - 1, L); break;
  }
  return x + L * (y + L * z);
}

/* Index of the bond between `site` and its neighbour along dir. */
static int bond_of(int site, int dir, int L) {
  int N = L * L * L;
  int d = dir / 2;
  if (dir % 2 == 0) return d * N + site;          /* bond from site to site+e_d */
  return d * N + neighbour(site, dir, L);         /* bond from site-e_d to site */
}

static int colour_of(int site, int L) {
  int x = site % L, y = (site / L) % L, z = site / (L * L);
  return (x + y + z) & 1;
}

/* Colour-major rank of every site, by counting (no closed form). */
void pao_colour_major(int L, int32_t* cm_out) {
  int N = L * L * L;
  int n0 = 0;
  for (int s = 0; s < N; ++s) n0 += (colour_of(s, L) == 0);
  int next0 = 0, next1 = n0;
  for (int s = 0; s < N; ++s) {
    if (colour_of(s, L) == 0) cm_out[s] = next0++;
    else cm_out[s] = next1++;
  }
}

void pao_neighbours(int L, int32_t* nbr_out /* N*6 */, int32_t* bond_out /* N*6 */) {
  int N = L * L * L;
  for (int s = 0; s < N; ++s)
    for (int dir = 0; dir < 6; ++dir) {
      nbr_out[s * 6 + dir] = neighbour(s, dir, L);
      bond_out[s * 6 + dir] = bond_of(s, dir, L);
    }
}

/* ------------------------------------------------------------------------ */
/* Energy.  With +-1 couplings the energy of a configuration is an integer: */
/* U = number of unsatisfied bonds (J_b s_i s_j = -1), E = 2U - 3N.           */
/* ------------------------------------------------------------------------ */
static int32_t unsatisfied_bonds(const int8_t* s, const int8_t* J, int L) {
  int N = L * L * L;
  int32_t U = 0;
  for (int site = 0; site < N; ++site)
    for (int d = 0; d < 3; ++d) {
      int other = neighbour(site, 2 * d, L);
      if ((int)J[d * N + site] * (int)s[site] * (int)s[other] < 0) ++U;
    }
  return U;
}

void pao_energy(int L, const int8_t* J, const int8_t* spins, int64_t R, int32_t* U_out) {
  int N = L * L * L;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < R; ++r) U_out[r] = unsatisfied_bonds(spins + r * N, J, L);
}

/* ------------------------------------------------------------------------ */
/* Initial population (Sec. II): R independent replicas drawn uniformly at  */
/* beta = 0, labelled 0..R-1 (each replica is its own family).               */
/* Spin of replica r at site: bit 31 of word (site & 3) of                   */
/* Philox(seed; r, site >> 2, 0, TAG_INIT); bit 0 -> +1, bit 1 -> -1.        */
/* ------------------------------------------------------------------------ */
void pao_init(int L, const int8_t* J, int64_t R, uint64_t seed, int8_t* spins_out,
              int32_t* U_out, uint32_t* family_out) {
  int N = L * L * L;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < R; ++r) {
    int8_t* s = spins_out + r * N;
    for (int site = 0; site < N; ++site) {
      uint32_t w = draw_word(seed, (uint32_t)r, (uint32_t)(site >> 2), 0u, TAG_INIT, site & 3);
      s[site] = (w >> 31) ? (int8_t)-1 : (int8_t)1;
    }
    U_out[r] = unsatisfied_bonds(s, J, L);
    family_out[r] = (uint32_t)r;
  }
}

/* ------------------------------------------------------------------------ */
/* Metropolis acceptance thresholds at inverse temperature beta: a move that */
/* raises the energy by dE > 0 is accepted with probability exp(-beta dE),  */
/* realised as  word < thr[dE]  with thr = floor(2^32 exp(-beta dE)).         */
/* dE is 4, 8 or 12 for +-J couplings on the cubic lattice.                  */
/* ------------------------------------------------------------------------ */
void pao_thresholds(double beta, uint64_t thr_out[3]) {
  for (int i = 0; i < 3; ++i) {
    double dE = (double)(4 * (i + 1));
    thr_out[i] = (uint64_t)floor(ldexp(exp(-beta * dE), 32));
  }
}

/* ------------------------------------------------------------------------ */
/* Metropolis sweeps (Sec. II: the MCMC step of PA; the variant is ours).   */
/* A sweep visits colour 0 then colour 1; within a colour, sites in          */
/* lexicographic order, each updated in place.  For even L same-colour sites */
/* never touch, so this equals a simultaneous checkerboard update.           */
/* The draw for (replica slot r, sweep t, site) is word (cm & 3) of          */
/* Philox(seed; r, t, cm >> 2, TAG_MET); it is needed only when dE > 0.      */
/* The population sweep counter t advances by one after every full sweep.    */
/* U is updated incrementally: U += dE/2 on every accepted flip.             */
/* ------------------------------------------------------------------------ */
/* Sweeps of one replica held in s[0..N) that sits in population slot `slot`. */
static void sweep_one(int L, const int8_t* J, const int32_t* cm, const int32_t* nb,
                      const int32_t* bd, int8_t* s, int32_t* U, uint32_t slot, uint64_t seed,
                      const uint64_t thr[3], uint32_t t0, int n_sweeps) {
  int N = L * L * L;
  int32_t u = *U;
  for (int sw = 0; sw < n_sweeps; ++sw) {
    uint32_t t = t0 + (uint32_t)sw;
    for (int colour = 0; colour < 2; ++colour) {
      for (int site = 0; site < N; ++site) {
        if (colour_of(site, L) != colour) continue;
        int h = 0;
        for (int dir = 0; dir < 6; ++dir)
          h += (int)J[bd[site * 6 + dir]] * (int)s[nb[site * 6 + dir]];
        int dE = 2 * (int)s[site] * h;
        int accept;
        if (dE <= 0) {
          accept = 1;
        } else {
          uint32_t x = draw_word(seed, slot, t, (uint32_t)(cm[site] >> 2), TAG_MET, cm[site] & 3);
          accept = (uint64_t)x < thr[dE / 4 - 1];
        }
        if (accept) {
          s[site] = (int8_t)(-s[site]);
          u += dE / 2;
        }
      }
    }
  }
  *U = u;
}

/* All replicas of a population: replica r sits in slot r. */
void pao_sweep(int L, const int8_t* J, int8_t* spins, int32_t* U, int64_t R_tilde,
               uint64_t seed, const uint64_t thr[3], uint32_t t0, int n_sweeps) {
  int N = L * L * L;
  /* lattice tables, filled once: neighbour site and bond of every direction */
  int32_t* cm = (int32_t*)malloc(sizeof(int32_t) * N);
  int32_t* nb = (int32_t*)malloc(sizeof(int32_t) * N * 6);
  int32_t* bd = (int32_t*)malloc(sizeof(int32_t) * N * 6);
  pao_colour_major(L, cm);
  pao_neighbours(L, nb, bd);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < R_tilde; ++r)
    sweep_one(L, J, cm, nb, bd, spins + r * N, U + r, (uint32_t)r, seed, thr, t0, n_sweeps);
  free(cm);
  free(nb);
  free(bd);
}

/* Selected replicas: replica i (row i of spins) sits in slot slots[i]. */
void pao_sweep_slots(int L, const int8_t* J, int8_t* spins, int32_t* U, int64_t n,
                     const uint32_t* slots, uint64_t seed, const uint64_t thr[3], uint32_t t0,
                     int n_sweeps) {
  int N = L * L * L;
  int32_t* cm = (int32_t*)malloc(sizeof(int32_t) * N);
  int32_t* nb = (int32_t*)malloc(sizeof(int32_t) * N * 6);
  int32_t* bd = (int32_t*)malloc(sizeof(int32_t) * N * 6);
  pao_colour_major(L, cm);
  pao_neighbours(L, nb, bd);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    sweep_one(L, J, cm, nb, bd, spins + i * N, U + i, slots[i], seed, thr, t0, n_sweeps);
  free(cm);
  free(nb);
  free(bd);
}

/* ------------------------------------------------------------------------ */
/* Energy histogram: h_j = number of replicas with U = j, j = 0..3N.          */
/* With integer energies the sum in the normaliser Q (Eq. 2) regroups by    */
/* level.                                                                    */
/* ------------------------------------------------------------------------ */
void pao_histogram(const int32_t* U, int64_t R_tilde, int n_levels, uint32_t* h_out) {
  memset(h_out, 0, sizeof(uint32_t) * (size_t)n_levels);
  for (int64_t i = 0; i < R_tilde; ++i) h_out[U[i]] += 1;
}

/* ------------------------------------------------------------------------ */
/* Resampling table for the step beta -> beta + dbeta (Sec. II, Eqs. 1-2).  */
/*   j_min = lowest occupied level (reference energy, avoids FP overflow;   */
/*           it cancels in tau)                                              */
/*   w_j   = exp(-dbeta * 2 (j - j_min))          (= e^{-dbeta (E_j - E_min)})*/
/*   S     = sum over occupied j, ascending, of h_j w_j                      */
/*   tau_j = R w_j / S                            (Eq. 1 with Eq. 2 inserted) */
/*   ln Q  = ln S - ln R~ - dbeta E_min           (Eq. 2, shifted back)       */
/* Copy-count split of tau_j: floor fl_j and an integer threshold             */
/*   T_j = ceil(frac(tau_j) 2^53), so that u53 < T_j  <=>  u < frac(tau_j).   */
/* Levels below j_min get fl = T = 0 (no replica sits there).                */
/* Returns j_min, or -1 for an empty histogram.                              */
/* ------------------------------------------------------------------------ */
int pao_table(const uint32_t* h, int n_levels, int N, uint32_t R, uint32_t R_tilde,
              double dbeta, uint32_t* fl_out, uint64_t* T_out, double* tau_out,
              double* lnQ_out) {
  int jmin = -1;
  for (int j = 0; j < n_levels; ++j)
    if (h[j] > 0) { jmin = j; break; }
  if (jmin < 0) return -1;
  double S = 0.0;
  for (int j = jmin; j < n_levels; ++j) {
    if (h[j] == 0) continue;
    double w = exp(-dbeta * (double)(2 * (j - jmin)));
    S = S + (double)h[j] * w;
  }
  for (int j = 0; j < n_levels; ++j) {
    if (j < jmin) {
      fl_out[j] = 0; T_out[j] = 0;
      if (tau_out) tau_out[j] = 0.0;
      continue;
    }
    double w = exp(-dbeta * (double)(2 * (j - jmin)));
    double tau = ((double)R * w) / S;
    uint64_t fl = (uint64_t)floor(tau);
    double fr = tau - (double)fl;
    fl_out[j] = (uint32_t)fl;
    T_out[j] = (uint64_t)ceil(ldexp(fr, 53));
    if (tau_out) tau_out[j] = tau;
  }
  *lnQ_out = log(S) - log((double)R_tilde) - dbeta * (double)(2 * jmin - 3 * N);
  return jmin;
}

/* ------------------------------------------------------------------------ */
/* Nearest-integer copy counts (Sec. II): n_i = floor(tau_i) with           */
/* probability ceil(tau_i) - tau_i, else ceil(tau_i).  The uniform is a     */
/* 53-bit integer u53 from words 0 and 1 of Philox(seed; i, k, 0, TAG_RES),  */
/* i = current slot, k = resampling step index; the extra copy is taken iff */
/* u53 < T_j (strict, so an integer tau never gets one).                     */
/* ------------------------------------------------------------------------ */
void pao_copy_counts(const int32_t* U, int64_t R_tilde, const uint32_t* fl, const uint64_t* T,
                     uint64_t seed, uint32_t step, uint32_t* n_out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < R_tilde; ++i) {
    uint32_t ctr[4] = {(uint32_t)i, step, 0u, TAG_RES};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    pao_philox(ctr, key, out);
    uint64_t u53 = ((uint64_t)out[0] << 21) | (uint64_t)(out[1] >> 11);
    int j = U[i];
    n_out[i] = fl[j] + (u53 < T[j] ? 1u : 0u);
  }
}

/* ------------------------------------------------------------------------ */
/* Copy / eliminate (Sec. II): replica i is copied n_i times; its copies    */
/* take consecutive new slots starting at offset_i = sum_{i'<i} n_i', so the */
/* new population keeps the old order and every copy inherits the family    */
/* label of its ancestor.  Returns the new population size, or -1 if it     */
/* exceeds `capacity` (the old population is then left untouched).          */
/* ------------------------------------------------------------------------ */
int64_t pao_copy_eliminate(int L, const uint32_t* n, int64_t R_tilde, int64_t capacity,
                           const int8_t* spins_old, const int32_t* U_old,
                           const uint32_t* fam_old, int8_t* spins_new, int32_t* U_new,
                           uint32_t* fam_new, uint64_t* offsets_out) {
  int N = L * L * L;
  uint64_t total = 0;
  for (int64_t i = 0; i < R_tilde; ++i) {
    if (offsets_out) offsets_out[i] = total;
    total += n[i];
  }
  if ((int64_t)total > capacity) return -1;
  uint64_t dst = 0;
  for (int64_t i = 0; i < R_tilde; ++i) {
    for (uint32_t c = 0; c < n[i]; ++c) {
      memcpy(spins_new + dst * N, spins_old + i * N, (size_t)N);
      U_new[dst] = U_old[i];
      fam_new[dst] = fam_old[i];
      ++dst;
    }
  }
  return (int64_t)total;
}

/* ------------------------------------------------------------------------ */
/* Culling fraction (Sec. III.C): eps R = sum over replicas with tau < 1 of */
/* (1 - tau), evaluated from the histogram with tau_j exactly as in         */
/* pao_table (same j_min shift, same ascending sum).                         */
/* ------------------------------------------------------------------------ */
double pao_culling_fraction(const uint32_t* h, int n_levels, uint32_t R, double dbeta) {
  int jmin = -1;
  for (int j = 0; j < n_levels; ++j)
    if (h[j] > 0) { jmin = j; break; }
  if (jmin < 0) return 0.0;
  double S = 0.0;
  for (int j = jmin; j < n_levels; ++j) {
    if (h[j] == 0) continue;
    double w = exp(-dbeta * (double)(2 * (j - jmin)));
    S = S + (double)h[j] * w;
  }
  double acc = 0.0;
  for (int j = jmin; j < n_levels; ++j) {
    if (h[j] == 0) continue;
    double w = exp(-dbeta * (double)(2 * (j - jmin)));
    double tau = ((double)R * w) / S;
    if (tau < 1.0) acc = acc + (double)h[j] * (1.0 - tau);
  }
  return acc / (double)R;
}

/* ------------------------------------------------------------------------ */
/* Constant-culling step (Sec. III.C and Sec. IV.B: a schedule that culls a */
/* fixed fraction per step), by the bisection of pao_choose_dbeta_unit with */
/* the +-J level width 2.                                                   */
/* ------------------------------------------------------------------------ */
int pao_choose_dbeta_unit(const uint32_t* h, int n_levels, double unit, uint32_t R,
                          double eps_target, double rem, double* dbeta_out, int* reached_end);

int pao_choose_dbeta(const uint32_t* h, int n_levels, uint32_t R, double eps_target,
                     double rem, double* dbeta_out, int* reached_end) {
  return pao_choose_dbeta_unit(h, n_levels, 2.0, R, eps_target, rem, dbeta_out, reached_end);
}

/* ------------------------------------------------------------------------ */
/* Family statistic (Sec. III.A, rho_t): sum over family labels f of eta_f^2*/
/* where eta_f counts the replicas carrying label f.  Labels are < R.       */
/* ------------------------------------------------------------------------ */
uint64_t pao_sum_eta2(const uint32_t* fam, int64_t R_tilde, uint32_t R) {
  uint64_t* eta = (uint64_t*)calloc((size_t)R, sizeof(uint64_t));
  for (int64_t i = 0; i < R_tilde; ++i) eta[fam[i]] += 1;
  uint64_t acc = 0;
  for (uint32_t f = 0; f < R; ++f) acc += eta[f] * eta[f];
  free(eta);
  return acc;
}

/* Family-size distribution: count_out[e] = number of labels with eta = e,   */
/* for e < max_eta; larger families are added to the last bin.              */
void pao_family_sizes(const uint32_t* fam, int64_t R_tilde, uint32_t R, int max_eta,
                      uint64_t* count_out) {
  uint64_t* eta = (uint64_t*)calloc((size_t)R, sizeof(uint64_t));
  for (int64_t i = 0; i < R_tilde; ++i) eta[fam[i]] += 1;
  memset(count_out, 0, sizeof(uint64_t) * (size_t)max_eta);
  for (uint32_t f = 0; f < R; ++f) {
    uint64_t e = eta[f];
    if (e >= (uint64_t)max_eta) e = (uint64_t)max_eta - 1;
    count_out[e] += 1;
  }
  free(eta);
}

/* ------------------------------------------------------------------------ */
/* Spin overlap (Sec. II.A): q = (1/N) sum_n s1_n s2_n between replica slot */
/* i of population A and slot i of population B (independent populations,  */
/* same couplings), for i < min(R~_A, R~_B).  With d = number of sites where */
/* they differ, q = 1 - 2d/N; the bin is round-half-up of 64 (1+q)/2, i.e.  */
/* (128 (N - d) + N) / (2N) in integer division: 65 bins over [-1, 1].       */
/* ------------------------------------------------------------------------ */
void pao_overlap_hist(int N, const int8_t* spins_a, int64_t Ra, const int8_t* spins_b,
                      int64_t Rb, uint64_t* hist65_out, uint32_t* d_out) {
  int64_t n = Ra < Rb ? Ra : Rb;
  memset(hist65_out, 0, sizeof(uint64_t) * 65);
  for (int64_t i = 0; i < n; ++i) {
    int d = 0;
    for (int site = 0; site < N; ++site) d += spins_a[i * N + site] != spins_b[i * N + site];
    if (d_out) d_out[i] = (uint32_t)d;
    int bin = (128 * (N - d) + N) / (2 * N);
    hist65_out[bin] += 1;
  }
}

/* ------------------------------------------------------------------------ */
/* Link overlap (Sec. II.A): for replica i of population a and replica i of  */
/* population b, q_l = (1/N_b) sum over the N_b = 3N bonds <n,m> of          */
/* s^a_n s^a_m s^b_n s^b_m.  Each term is +1 or -1, so the sum is N_b - 2 D  */
/* with D the number of bonds whose term is -1; D_out[i] receives D.  The    */
/* bonds are those of the periodic cubic lattice: every site with its +x, +y */
/* and +z neighbour (site = x + L (y + L z)).                                 */
/* ------------------------------------------------------------------------ */
void pao_link_overlap(int L, const int8_t* spins_a, int64_t Ra, const int8_t* spins_b, int64_t Rb,
                      uint32_t* D_out) {
  int64_t n = Ra < Rb ? Ra : Rb;
  int N = L * L * L;
  for (int64_t i = 0; i < n; ++i) {
    const int8_t* sa = spins_a + i * N;
    const int8_t* sb = spins_b + i * N;
    uint32_t D = 0;
    for (int z = 0; z < L; ++z)
      for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
          int site = x + L * (y + L * z);
          int nb[3] = {(x + 1) % L + L * (y + L * z), x + L * ((y + 1) % L + L * z),
                       x + L * (y + L * ((z + 1) % L))};
          for (int d = 0; d < 3; ++d) {
            int m = nb[d];
            int term = sa[site] * sa[m] * sb[site] * sb[m];
            if (term < 0) D += 1;
          }
        }
    D_out[i] = D;
  }
}

/* ------------------------------------------------------------------------ */
/* Exact density of states for a small lattice (N <= 30) by enumerating all */
/* 2^N states in Gray-code order: consecutive states differ by one spin, so */
/* U changes by (number of that spin's bonds made unsatisfied) minus        */
/* (number made satisfied).  g_out has 3N + 1 entries, g_out[U] = number of */
/* states with U unsatisfied bonds.                                          */
/* ------------------------------------------------------------------------ */
int pao_density_of_states(int L, const int8_t* J, uint64_t* g_out) {
  int N = L * L * L;
  if (N > 30) return -1;
  int nb[30][6];
  int jb[30][6];
  for (int s = 0; s < N; ++s)
    for (int dir = 0; dir < 6; ++dir) {
      nb[s][dir] = neighbour(s, dir, L);
      jb[s][dir] = J[bond_of(s, dir, L)];
    }
  memset(g_out, 0, sizeof(uint64_t) * (size_t)(3 * N + 1));
  /* state: bit s set <=> spin s is -1.  Start from all +1. */
  uint32_t state = 0;
  int8_t s[30];
  for (int i = 0; i < N; ++i) s[i] = 1;
  int U = unsatisfied_bonds(s, J, L);
  g_out[U] += 1;
  uint64_t total = (uint64_t)1 << N;
  for (uint64_t g = 1; g < total; ++g) {
    int flip = __builtin_ctzll(g);
    /* bonds of `flip`: unsatisfied before the flip become satisfied, and the
     * other way round */
    int before = 0;
    for (int dir = 0; dir < 6; ++dir)
      before += (jb[flip][dir] * s[flip] * s[nb[flip][dir]] < 0);
    U += 6 - 2 * before;
    s[flip] = (int8_t)(-s[flip]);
    state ^= 1u << flip;
    g_out[U] += 1;
  }
  (void)state;
  return 0;
}

/* ======================================================================== */
/* Gaussian couplings (Sec. II.A: the paper draws J_nm from a unit normal).  */
/* Reading: J = k / 16 with k an integer in [-127, 127] (a unit normal       */
/* rounded to the nearest 1/16), so that every energy is an integer number  */
/* of quanta 1/16 and the annealing loop keeps integer energy levels.       */
/*   E16 = -sum_b k_b s_i s_j            (E = E16 / 16)                      */
/* Flipping s_i changes E16 by dE16 = 2 s_i sum_j k_ij s_j, an even integer */
/* with |dE16| <= 2 * 6 * 127.                                               */
/* ======================================================================== */
static int32_t energy16(const int8_t* s, const int8_t* K, int L) {
  int N = L * L * L;
  int32_t e = 0;
  for (int d = 0; d < 3; ++d)
    for (int site = 0; site < N; ++site) {
      int other = neighbour(site, 2 * d, L);
      e -= (int32_t)K[d * N + site] * (int32_t)s[site] * (int32_t)s[other];
    }
  return e;
}

void pao_g_energy(int L, const int8_t* K, const int8_t* spins, int64_t R, int32_t* E16_out) {
  int N = L * L * L;
  for (int64_t r = 0; r < R; ++r) E16_out[r] = energy16(spins + r * N, K, L);
}

/* thr[d] = floor(2^32 exp(-beta d / 16)) for d = 0..dEmax (thr[0] = 2^32): */
/* a move raising E16 by d > 0 is taken iff its draw is below thr[d].       */
void pao_g_thresholds(double beta, int dEmax, uint64_t* thr_out) {
  for (int d = 0; d <= dEmax; ++d)
    thr_out[d] = (uint64_t)floor(ldexp(exp(-beta * ((double)d / 16.0)), 32));
}

/* Sweeps of one replica (same visiting order and draws as sweep_one). */
static void g_sweep_one(int L, const int8_t* K, const int32_t* cm, const int32_t* nb,
                        const int32_t* bd, int8_t* s, int32_t* E16, uint32_t slot, uint64_t seed,
                        const uint64_t* thr, uint32_t t0, int n_sweeps) {
  int N = L * L * L;
  int32_t e = *E16;
  for (int sw = 0; sw < n_sweeps; ++sw) {
    uint32_t t = t0 + (uint32_t)sw;
    for (int colour = 0; colour < 2; ++colour) {
      for (int site = 0; site < N; ++site) {
        if (colour_of(site, L) != colour) continue;
        int h = 0;
        for (int dir = 0; dir < 6; ++dir)
          h += (int)K[bd[site * 6 + dir]] * (int)s[nb[site * 6 + dir]];
        int dE = 2 * (int)s[site] * h;
        int accept;
        if (dE <= 0) {
          accept = 1;
        } else {
          uint32_t x = draw_word(seed, slot, t, (uint32_t)(cm[site] >> 2), TAG_MET, cm[site] & 3);
          accept = (uint64_t)x < thr[dE];
        }
        if (accept) {
          s[site] = (int8_t)(-s[site]);
          e += dE;
        }
      }
    }
  }
  *E16 = e;
}

void pao_g_sweep_slots(int L, const int8_t* K, int8_t* spins, int32_t* E16, int64_t n,
                       const uint32_t* slots, uint64_t seed, const uint64_t* thr, uint32_t t0,
                       int n_sweeps) {
  int N = L * L * L;
  int32_t* cm = (int32_t*)malloc(sizeof(int32_t) * N);
  int32_t* nb = (int32_t*)malloc(sizeof(int32_t) * N * 6);
  int32_t* bd = (int32_t*)malloc(sizeof(int32_t) * N * 6);
  pao_colour_major(L, cm);
  pao_neighbours(L, nb, bd);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    g_sweep_one(L, K, cm, nb, bd, spins + i * N, E16 + i, slots ? slots[i] : (uint32_t)i, seed,
                thr, t0, n_sweeps);
  free(cm);
  free(nb);
  free(bd);
}

/* Resampling table with energy levels of width `unit` (Sec. II, Eqs. 1-2): */
/* level j has energy unit * (E_lo + j); otherwise as pao_table:            */
/*   w_j = exp(-dbeta * (unit * (j - j_min))), S = ascending sum of h_j w_j, */
/*   tau_j = R w_j / S, fl_j, T_j as in pao_table,                           */
/*   ln Q = ln S - ln R~ - dbeta * unit * (E_lo + j_min).                    */
int pao_table_unit(const uint32_t* h, int n_levels, double unit, int64_t E_lo, uint32_t R,
                   uint32_t R_tilde, double dbeta, uint32_t* fl_out, uint64_t* T_out,
                   double* tau_out, double* lnQ_out) {
  int jmin = -1;
  for (int j = 0; j < n_levels; ++j)
    if (h[j] > 0) { jmin = j; break; }
  if (jmin < 0) return -1;
  double S = 0.0;
  for (int j = jmin; j < n_levels; ++j) {
    if (h[j] == 0) continue;
    double w = exp(-dbeta * (unit * (double)(j - jmin)));
    S = S + (double)h[j] * w;
  }
  for (int j = 0; j < n_levels; ++j) {
    if (j < jmin) {
      fl_out[j] = 0; T_out[j] = 0;
      if (tau_out) tau_out[j] = 0.0;
      continue;
    }
    double w = exp(-dbeta * (unit * (double)(j - jmin)));
    double tau = ((double)R * w) / S;
    uint64_t fl = (uint64_t)floor(tau);
    double fr = tau - (double)fl;
    fl_out[j] = (uint32_t)fl;
    T_out[j] = (uint64_t)ceil(ldexp(fr, 53));
    if (tau_out) tau_out[j] = tau;
  }
  *lnQ_out = log(S) - log((double)R_tilde) - dbeta * (unit * (double)(E_lo + jmin));
  return jmin;
}

/* Culling fraction with levels of width `unit` (as pao_culling_fraction). */
double pao_culling_fraction_unit(const uint32_t* h, int n_levels, double unit, uint32_t R,
                                 double dbeta) {
  int jmin = -1;
  for (int j = 0; j < n_levels; ++j)
    if (h[j] > 0) { jmin = j; break; }
  if (jmin < 0) return 0.0;
  double S = 0.0;
  for (int j = jmin; j < n_levels; ++j) {
    if (h[j] == 0) continue;
    double w = exp(-dbeta * (unit * (double)(j - jmin)));
    S = S + (double)h[j] * w;
  }
  double acc = 0.0;
  for (int j = jmin; j < n_levels; ++j) {
    if (h[j] == 0) continue;
    double w = exp(-dbeta * (unit * (double)(j - jmin)));
    double tau = ((double)R * w) / S;
    if (tau < 1.0) acc = acc + (double)h[j] * (1.0 - tau);
  }
  return acc / (double)R;
}

/* Constant-culling step with levels of width `unit` (Sec. III.C).  Our     */
/* reading: bisect dbeta on [0, rem] so that eps(dbeta) <= eps_target, 64   */
/* halvings with mid = lo + (hi - lo)/2, keeping the lower end; if the whole */
/* remaining range already culls no more than eps_target, take it.  Returns */
/* 0, or -1 when even dbeta = 0 culls more than eps_target.                 */
/* ------------------------------------------------------------------------ */
int pao_choose_dbeta_unit(const uint32_t* h, int n_levels, double unit, uint32_t R,
                          double eps_target, double rem, double* dbeta_out, int* reached_end) {
  if (pao_culling_fraction_unit(h, n_levels, unit, R, 0.0) > eps_target) return -1;
  if (pao_culling_fraction_unit(h, n_levels, unit, R, rem) <= eps_target) {
    *dbeta_out = rem;
    *reached_end = 1;
    return 0;
  }
  double lo = 0.0, hi = rem;
  for (int it = 0; it < 64; ++it) {
    double mid = lo + 0.5 * (hi - lo);
    if (pao_culling_fraction_unit(h, n_levels, unit, R, mid) <= eps_target) lo = mid;
    else hi = mid;
  }
  *dbeta_out = lo;
  *reached_end = 0;
  return 0;
}

/* Exact density of states over E16 (N <= 30), Gray-code enumeration:      */
/* g_out[E16 + off] counts the states with energy E16, off = 3 * 127 * N.    */
int pao_g_density_of_states(int L, const int8_t* K, uint64_t* g_out) {
  int N = L * L * L;
  if (N > 30) return -1;
  int nb[30][6];
  int kb[30][6];
  for (int s = 0; s < N; ++s)
    for (int dir = 0; dir < 6; ++dir) {
      nb[s][dir] = neighbour(s, dir, L);
      kb[s][dir] = K[bond_of(s, dir, L)];
    }
  const int off = 3 * 127 * N;
  memset(g_out, 0, sizeof(uint64_t) * (size_t)(2 * off + 1));
  int8_t s[30];
  for (int i = 0; i < N; ++i) s[i] = 1;
  int e = energy16(s, K, L);
  g_out[e + off] += 1;
  uint64_t total = (uint64_t)1 << N;
  for (uint64_t g = 1; g < total; ++g) {
    int f = __builtin_ctzll(g);
    int h = 0;
    for (int dir = 0; dir < 6; ++dir) h += kb[f][dir] * s[nb[f][dir]];
    e += 2 * s[f] * h;
    s[f] = (int8_t)(-s[f]);
    g_out[e + off] += 1;
  }
  return 0;
}

/* ======================================================================== */
/* Gaussian couplings, continuous (Sec. II.A: J_nm drawn from a unit        */
/* normal).                                                                  */
/*                                                                           */
/* Reading: every coupling is an FP64 number on the grid 2^-32 with          */
/* |J| < 8 (the caller rounds a unit normal to the nearest grid point; a     */
/* draw beyond 8 sd has probability 1e-15 per bond).  Every energy is then a */
/* sum of at most 3N <= 12288 grid numbers below 8 in size: |E| < 2^17, a    */
/* multiple of 2^-32, so every partial sum fits in 49 bits and FP64 adds it  */
/* exactly, in any order.  Energies and energy changes are therefore exact.  */
/*                                                                           */
/* Floating point enters in three places, each written out below so that a   */
/* second implementation of the same steps gets the same bits:               */
/*   pao_r_exp     exp(x), x <= 0, by a fixed sequence of IEEE operations     */
/*   fixed-point sums of weights (S of Eq. 2, the culled mass of Sec. III.C)  */
/*   the copy-count split (as for the other models)                           */
/* ======================================================================== */

/* exp(x) for x <= 0.  Cody and Waite's argument reduction (Software Manual   */
/* for the Elementary Functions, 1980) with a Taylor polynomial:              */
/*   x < -708          -> 0 (below 2^-1021; no weight or threshold uses it)   */
/*   k  = x * log2(e), rounded to the nearest integer (ties to even)         */
/*   r  = fma(-k, ln2_hi, x);  r = fma(-k, ln2_lo, r)    (|r| <= 0.3466)      */
/*   p  = sum_{n=0..13} r^n / n!   by Horner's rule, one fma per degree      */
/*   exp(x) = p 2^k                                                           */
/* ln2_hi is ln 2 rounded to FP64, ln2_lo the rounded remainder, log2(e) and  */
/* 1/n! rounded to FP64.  The truncated series errs by r^14/14! < 5e-18,     */
/* below half an ulp of p; the result is within about one ulp of exp(x).     */
/* ------------------------------------------------------------------------ */
double pao_r_exp(double x) {
  if (x < -708.0) return 0.0;
  double k = nearbyint(x * 0x1.71547652b82fep+0);
  double r = fma(-k, 0x1.62e42fefa39efp-1, x);
  r = fma(-k, 0x1.abc9e3b39803fp-56, r);
  double p = 1.0 / 6227020800.0;               /* 1/13! */
  p = fma(p, r, 1.0 / 479001600.0);            /* 1/12! */
  p = fma(p, r, 1.0 / 39916800.0);             /* 1/11! */
  p = fma(p, r, 1.0 / 3628800.0);              /* 1/10! */
  p = fma(p, r, 1.0 / 362880.0);               /* 1/9!  */
  p = fma(p, r, 1.0 / 40320.0);                /* 1/8!  */
  p = fma(p, r, 1.0 / 5040.0);                 /* 1/7!  */
  p = fma(p, r, 1.0 / 720.0);                  /* 1/6!  */
  p = fma(p, r, 1.0 / 120.0);                  /* 1/5!  */
  p = fma(p, r, 1.0 / 24.0);                   /* 1/4!  */
  p = fma(p, r, 1.0 / 6.0);                    /* 1/3!  */
  p = fma(p, r, 0.5);                          /* 1/2!  */
  p = fma(p, r, 1.0);                          /* 1/1!  */
  p = fma(p, r, 1.0);                          /* 1/0!  */
  return ldexp(p, (int)k);
}

void pao_r_exp_many(const double* x, int64_t n, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = pao_r_exp(x[i]);
}

/* E = -sum_b J_b s_i s_j over the 3N bonds (exact, see above). */
static double energy_r(const int8_t* s, const double* J, int L) {
  int N = L * L * L;
  double e = 0.0;
  for (int d = 0; d < 3; ++d)
    for (int site = 0; site < N; ++site) {
      int other = neighbour(site, 2 * d, L);
      e -= J[d * N + site] * (double)(s[site] * s[other]);
    }
  return e;
}

void pao_r_energy(int L, const double* J, const int8_t* spins, int64_t R, double* E_out) {
  int N = L * L * L;
  for (int64_t r = 0; r < R; ++r) E_out[r] = energy_r(spins + r * N, J, L);
}

/* Metropolis threshold of a move raising the energy by dE at inverse       */
/* temperature beta: 2^32 (always taken) for dE <= 0, else                  */
/* floor(2^32 pao_r_exp(-beta dE)); the move is taken iff its draw is below. */
uint64_t pao_r_threshold(double beta, double dE) {
  if (dE <= 0.0) return (uint64_t)1 << 32;
  return (uint64_t)floor(ldexp(pao_r_exp(-beta * dE), 32));
}

/* Sweeps of one replica: the visiting order and draws of sweep_one, with    */
/* dE = 2 s_i sum_j J_ij s_j in FP64 (exact) and the threshold above.       */
static void r_sweep_one(int L, const double* J, const int32_t* cm, const int32_t* nb,
                        const int32_t* bd, int8_t* s, double* E, uint32_t slot, uint64_t seed,
                        double beta, uint32_t t0, int n_sweeps) {
  int N = L * L * L;
  double e = *E;
  for (int sw = 0; sw < n_sweeps; ++sw) {
    uint32_t t = t0 + (uint32_t)sw;
    for (int colour = 0; colour < 2; ++colour) {
      for (int site = 0; site < N; ++site) {
        if (colour_of(site, L) != colour) continue;
        double h = 0.0;
        for (int dir = 0; dir < 6; ++dir)
          h += J[bd[site * 6 + dir]] * (double)s[nb[site * 6 + dir]];
        double dE = 2.0 * (double)s[site] * h;
        int accept;
        if (dE <= 0.0) {
          accept = 1;
        } else {
          uint32_t x = draw_word(seed, slot, t, (uint32_t)(cm[site] >> 2), TAG_MET, cm[site] & 3);
          accept = (uint64_t)x < pao_r_threshold(beta, dE);
        }
        if (accept) {
          s[site] = (int8_t)(-s[site]);
          e += dE;
        }
      }
    }
  }
  *E = e;
}

void pao_r_sweep_slots(int L, const double* J, int8_t* spins, double* E, int64_t n,
                       const uint32_t* slots, uint64_t seed, double beta, uint32_t t0,
                       int n_sweeps) {
  int N = L * L * L;
  int32_t* cm = (int32_t*)malloc(sizeof(int32_t) * N);
  int32_t* nb = (int32_t*)malloc(sizeof(int32_t) * N * 6);
  int32_t* bd = (int32_t*)malloc(sizeof(int32_t) * N * 6);
  pao_colour_major(L, cm);
  pao_neighbours(L, nb, bd);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    r_sweep_one(L, J, cm, nb, bd, spins + i * N, E + i, slots ? slots[i] : (uint32_t)i, seed,
                beta, t0, n_sweeps);
  free(cm);
  free(nb);
  free(bd);
}

/* Resampling weights (Eq. 1): w_i = pao_r_exp(-(dbeta (E_i - E_min))),     */
/* E_min the population's lowest energy (reference shift; it cancels in     */
/* tau), so 0 <= w_i <= 1 and the lowest replica has weight 1.              */
void pao_r_weights(const double* E, int64_t n, double dbeta, double E_min, double* w_out) {
  for (int64_t i = 0; i < n; ++i) w_out[i] = pao_r_exp(-(dbeta * (E[i] - E_min)));
}

/* Fixed-point sum of values in [0, 1]: sum_i floor(v_i 2^96), exactly, as a */
/* 128-bit integer (out[0] low word, out[1] high word; R <= 2^31 terms keep */
/* it below 2^127).  The caller rounds it once to FP64 (nearest, ties to    */
/* even) and scales by 2^-96.  Reading: the normaliser S of Eq. 2 and the    */
/* culled mass of Sec. III.C are such sums; truncating each term moves the   */
/* total by less than R 2^-96, and the integer sum has no order.             */
void pao_r_fixsum96(const double* v, int64_t n, uint64_t out[2]) {
  unsigned __int128 acc = 0;
  for (int64_t i = 0; i < n; ++i) {
    double x = v[i];
    if (x == 0.0) continue;
    int e;
    double m = frexp(x, &e);                       /* x = m 2^e, 1/2 <= m < 1 */
    uint64_t M = (uint64_t)ldexp(m, 53);           /* x = M 2^(e - 53), exact */
    int sh = e - 53 + 96;
    if (sh >= 0) acc += (unsigned __int128)M << sh;
    else if (sh > -64) acc += (unsigned __int128)(M >> -sh);
  }
  out[0] = (uint64_t)acc;
  out[1] = (uint64_t)(acc >> 64);
}

/* Copy counts from per-replica weights (Sec. II, Eqs. 1-2):                */
/*   tau_i = (R w_i) / S,  fl_i = floor(tau_i),                              */
/*   T_i = ceil(frac(tau_i) 2^53),  n_i = fl_i + [u53 < T_i]                 */
/* with u53 drawn as in pao_copy_counts (slot i, step k).                    */
void pao_r_copy_counts(const double* w, int64_t R_tilde, uint32_t R, double S, uint64_t seed,
                       uint32_t step, uint32_t* n_out, double* tau_out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < R_tilde; ++i) {
    double tau = ((double)R * w[i]) / S;
    uint64_t fl = (uint64_t)floor(tau);
    double fr = tau - (double)fl;
    uint64_t T = (uint64_t)ceil(ldexp(fr, 53));
    uint32_t ctr[4] = {(uint32_t)i, step, 0u, TAG_RES};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    pao_philox(ctr, key, out);
    uint64_t u53 = ((uint64_t)out[0] << 21) | (uint64_t)(out[1] >> 11);
    n_out[i] = (uint32_t)fl + (u53 < T ? 1u : 0u);
    if (tau_out) tau_out[i] = tau;
  }
}

/* Culled mass terms (Sec. III.C): c_i = 1 - tau_i if tau_i < 1, else 0;    */
/* eps = (fixed-point sum of c_i) / R.                                       */
void pao_r_cull_terms(const double* w, int64_t R_tilde, uint32_t R, double S, double* c_out) {
  for (int64_t i = 0; i < R_tilde; ++i) {
    double tau = ((double)R * w[i]) / S;
    c_out[i] = tau < 1.0 ? 1.0 - tau : 0.0;
  }
}

/* Exact thermodynamics of a small lattice with real couplings (N <= 30):   */
/* Gray-code enumeration of all 2^N states, in 2^6 independent slices.      */
/* Pass 1 finds the ground-state energy E0 (exact); pass 2 sums, for every  */
/* beta, Z0 = sum exp(-beta (E - E0)), Z1 = sum (E - E0) exp(.), Z2 = sum   */
/* (E - E0)^2 exp(.) with the C library's exp.  Out (per beta):             */
/* lnZ = ln Z0 - beta E0, <E> = E0 + Z1/Z0, var E = Z2/Z0 - (Z1/Z0)^2.       */
int pao_r_exact_thermo(int L, const double* J, int n_beta, const double* betas,
                       double* lnZ_out, double* E_out, double* varE_out, double* E0_out) {
  int N = L * L * L;
  if (N > 30 || N < 7 || n_beta > 64) return -1;
  int nb[30][6];
  double jb[30][6];
  for (int s = 0; s < N; ++s)
    for (int dir = 0; dir < 6; ++dir) {
      nb[s][dir] = neighbour(s, dir, L);
      jb[s][dir] = J[bond_of(s, dir, L)];
    }
  const int SLICE_BITS = 6;
  const int low = N - SLICE_BITS;
  const uint64_t per = (uint64_t)1 << low;
  double e0_slice[64];
  double z[64][64][3];
  for (int pass = 0; pass < 2; ++pass) {
    double E0 = 0.0;
    if (pass == 1) {
      E0 = e0_slice[0];
      for (int sl = 1; sl < 64; ++sl)
        if (e0_slice[sl] < E0) E0 = e0_slice[sl];
      *E0_out = E0;
    }
#pragma omp parallel for schedule(dynamic)
    for (int sl = 0; sl < 64; ++sl) {
      int8_t s[30];
      for (int i = 0; i < N; ++i) s[i] = 1;
      for (int b = 0; b < SLICE_BITS; ++b)
        if ((sl >> b) & 1) s[low + b] = -1;
      double e = energy_r(s, J, L);
      double emin = e;
      double acc[64][3];
      memset(acc, 0, sizeof(acc));
      for (uint64_t g = 0; g < per; ++g) {
        if (g > 0) {
          int f = __builtin_ctzll(g);
          double h = 0.0;
          for (int dir = 0; dir < 6; ++dir) h += jb[f][dir] * (double)s[nb[f][dir]];
          e += 2.0 * (double)s[f] * h;
          s[f] = (int8_t)(-s[f]);
        }
        if (pass == 0) {
          if (e < emin) emin = e;
        } else {
          double d = e - E0;
          for (int k = 0; k < n_beta; ++k) {
            double x = exp(-betas[k] * d);
            acc[k][0] += x;
            acc[k][1] += d * x;
            acc[k][2] += d * d * x;
          }
        }
      }
      if (pass == 0) e0_slice[sl] = emin;
      else memcpy(z[sl], acc, sizeof(acc));
    }
    if (pass == 1) {
      for (int k = 0; k < n_beta; ++k) {
        double z0 = 0.0, z1 = 0.0, z2 = 0.0;
        for (int sl = 0; sl < 64; ++sl) {
          z0 += z[sl][k][0];
          z1 += z[sl][k][1];
          z2 += z[sl][k][2];
        }
        double m1 = z1 / z0;
        lnZ_out[k] = log(z0) - betas[k] * E0;
        E_out[k] = E0 + m1;
        varE_out[k] = z2 / z0 - m1 * m1;
      }
    }
  }
  return 0;
}
