"""CPU oracle for the population-annealing hot path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library ``paper_1711_02146_amd``; neither imports the other.

The arithmetic lives in ``pa_oracle.c`` (plain C, compiled with gcc,
``-ffp-contract=off``); this module binds it with ctypes and runs the
annealing loop of Sec. II of Amey & Machta (arXiv:1711.02146) step by step:

    resample beta_{k-1} -> beta_k   (Eqs. 1-2, nearest-integer copy counts,
                                     copy/eliminate with family labels)
    N_S Metropolis sweeps at beta_k (the MCMC step of Sec. II)
    measure                          (<E>, beta F from Eq. 9, rho_t of Sec. III.A)

The per-step scalars (<E>, beta F, rho_t) are formed here in Python floats,
which are IEEE doubles, one operation at a time in the order written.

Three coupling models: +-J (Population), Gaussian rounded to multiples of
1/16 (GaussPopulation, integer energy levels) and real Gaussian couplings on
the grid 2^-32 (GaussRealPopulation: exact FP64 energies, per-replica
weights, the normaliser and culled mass summed in fixed point).

Parity unpinned: the overlap bin convention and the denominator R of rho_t
(see pa_oracle.c) are checked between the oracle and the GPU only.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pa_oracle.c")
_LIB = os.path.join(_HERE, "libpa_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off"]


def build(force: bool = True) -> str:
    """Compile pa_oracle.c into libpa_oracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_c = ctypes


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_LIB)
    sig = {
        "pao_philox": (None, [_u32p, _u32p, _u32p]),
        "pao_make_couplings_pm": (None, [_c.c_uint64, _c.c_int, _i8p]),
        "pao_colour_major": (None, [_c.c_int, _i32p]),
        "pao_neighbours": (None, [_c.c_int, _i32p, _i32p]),
        "pao_energy": (None, [_c.c_int, _i8p, _i8p, _c.c_int64, _i32p]),
        "pao_init": (None, [_c.c_int, _i8p, _c.c_int64, _c.c_uint64, _i8p, _i32p, _u32p]),
        "pao_thresholds": (None, [_c.c_double, _u64p]),
        "pao_sweep": (None, [_c.c_int, _i8p, _i8p, _i32p, _c.c_int64, _c.c_uint64, _u64p,
                             _c.c_uint32, _c.c_int]),
        "pao_sweep_slots": (None, [_c.c_int, _i8p, _i8p, _i32p, _c.c_int64, _u32p, _c.c_uint64,
                                   _u64p, _c.c_uint32, _c.c_int]),
        "pao_histogram": (None, [_i32p, _c.c_int64, _c.c_int, _u32p]),
        "pao_table": (_c.c_int, [_u32p, _c.c_int, _c.c_int, _c.c_uint32, _c.c_uint32,
                                 _c.c_double, _u32p, _u64p, _f64p,
                                 _c.POINTER(_c.c_double)]),
        "pao_copy_counts": (None, [_i32p, _c.c_int64, _u32p, _u64p, _c.c_uint64, _c.c_uint32,
                                   _u32p]),
        "pao_copy_eliminate": (_c.c_int64, [_c.c_int, _u32p, _c.c_int64, _c.c_int64, _i8p, _i32p,
                                            _u32p, _i8p, _i32p, _u32p, _u64p]),
        "pao_culling_fraction": (_c.c_double, [_u32p, _c.c_int, _c.c_uint32, _c.c_double]),
        "pao_choose_dbeta": (_c.c_int, [_u32p, _c.c_int, _c.c_uint32, _c.c_double, _c.c_double,
                                        _c.POINTER(_c.c_double), _c.POINTER(_c.c_int)]),
        "pao_sum_eta2": (_c.c_uint64, [_u32p, _c.c_int64, _c.c_uint32]),
        "pao_family_sizes": (None, [_u32p, _c.c_int64, _c.c_uint32, _c.c_int, _u64p]),
        "pao_overlap_hist": (None, [_c.c_int, _i8p, _c.c_int64, _i8p, _c.c_int64, _u64p, _u32p]),
        "pao_link_overlap": (None, [_c.c_int, _i8p, _c.c_int64, _i8p, _c.c_int64, _u32p]),
        "pao_density_of_states": (_c.c_int, [_c.c_int, _i8p, _u64p]),
        "pao_g_energy": (None, [_c.c_int, _i8p, _i8p, _c.c_int64, _i32p]),
        "pao_g_thresholds": (None, [_c.c_double, _c.c_int, _u64p]),
        "pao_g_sweep_slots": (None, [_c.c_int, _i8p, _i8p, _i32p, _c.c_int64, _u32p,
                                     _c.c_uint64, _u64p, _c.c_uint32, _c.c_int]),
        "pao_table_unit": (_c.c_int, [_u32p, _c.c_int, _c.c_double, _c.c_int64, _c.c_uint32,
                                      _c.c_uint32, _c.c_double, _u32p, _u64p, _f64p,
                                      _c.POINTER(_c.c_double)]),
        "pao_culling_fraction_unit": (_c.c_double, [_u32p, _c.c_int, _c.c_double, _c.c_uint32,
                                                    _c.c_double]),
        "pao_choose_dbeta_unit": (_c.c_int, [_u32p, _c.c_int, _c.c_double, _c.c_uint32,
                                             _c.c_double, _c.c_double, _c.POINTER(_c.c_double),
                                             _c.POINTER(_c.c_int)]),
        "pao_g_density_of_states": (_c.c_int, [_c.c_int, _i8p, _u64p]),
        "pao_r_exp": (_c.c_double, [_c.c_double]),
        "pao_r_exp_many": (None, [_f64p, _c.c_int64, _f64p]),
        "pao_r_energy": (None, [_c.c_int, _f64p, _i8p, _c.c_int64, _f64p]),
        "pao_r_threshold": (_c.c_uint64, [_c.c_double, _c.c_double]),
        "pao_r_sweep_slots": (None, [_c.c_int, _f64p, _i8p, _f64p, _c.c_int64, _u32p,
                                     _c.c_uint64, _c.c_double, _c.c_uint32, _c.c_int]),
        "pao_r_weights": (None, [_f64p, _c.c_int64, _c.c_double, _c.c_double, _f64p]),
        "pao_r_fixsum96": (None, [_f64p, _c.c_int64, _u64p]),
        "pao_r_copy_counts": (None, [_f64p, _c.c_int64, _c.c_uint32, _c.c_double, _c.c_uint64,
                                     _c.c_uint32, _u32p, _f64p]),
        "pao_r_cull_terms": (None, [_f64p, _c.c_int64, _c.c_uint32, _c.c_double, _f64p]),
        "pao_r_exact_thermo": (_c.c_int, [_c.c_int, _f64p, _c.c_int, _f64p, _f64p, _f64p, _f64p,
                                          _c.POINTER(_c.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


# ---------------------------------------------------------------------------
# thin wrappers
# ---------------------------------------------------------------------------
def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 of counter (4 words) and key (2 words) -> 4 words."""
    out = np.zeros(4, np.uint32)
    lib().pao_philox(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def make_couplings_pm(L: int, coupling_seed: int) -> np.ndarray:
    """3 L^3 couplings +-1 drawn from Philox under the coupling seed (tag J)."""
    out = np.zeros(3 * L ** 3, np.int8)
    lib().pao_make_couplings_pm(int(coupling_seed), int(L), out)
    return out


def colour_major(L: int) -> np.ndarray:
    out = np.zeros(L ** 3, np.int32)
    lib().pao_colour_major(L, out)
    return out


def neighbours(L: int):
    N = L ** 3
    nb = np.zeros(N * 6, np.int32)
    bd = np.zeros(N * 6, np.int32)
    lib().pao_neighbours(L, nb, bd)
    return nb.reshape(N, 6), bd.reshape(N, 6)


def energy(L: int, J: np.ndarray, spins: np.ndarray) -> np.ndarray:
    spins = np.ascontiguousarray(spins, np.int8)
    R = spins.size // L ** 3
    U = np.zeros(R, np.int32)
    lib().pao_energy(L, np.ascontiguousarray(J, np.int8), spins, R, U)
    return U


def thresholds(beta: float) -> np.ndarray:
    out = np.zeros(3, np.uint64)
    lib().pao_thresholds(float(beta), out)
    return out


def sweep_slots(L: int, J: np.ndarray, spins: np.ndarray, U: np.ndarray, slots: np.ndarray,
                seed: int, beta: float, t0: int, n_sweeps: int):
    """Sweep selected replicas in place; row i sits in population slot slots[i]."""
    assert spins.dtype == np.int8 and spins.flags.c_contiguous
    assert U.dtype == np.int32 and U.flags.c_contiguous
    slots = np.ascontiguousarray(slots, np.uint32)
    lib().pao_sweep_slots(L, np.ascontiguousarray(J, np.int8), spins.reshape(-1), U, slots.size,
                          slots, seed, thresholds(beta), t0, n_sweeps)


def histogram(U: np.ndarray, n_levels: int) -> np.ndarray:
    h = np.zeros(n_levels, np.uint32)
    lib().pao_histogram(np.ascontiguousarray(U, np.int32), U.size, n_levels, h)
    return h


def table(h: np.ndarray, N: int, R: int, R_tilde: int, dbeta: float):
    """Resampling table (fl, T, tau, lnQ, jmin) for one step; see pa_oracle.c."""
    n = h.size
    fl = np.zeros(n, np.uint32)
    T = np.zeros(n, np.uint64)
    tau = np.zeros(n, np.float64)
    lnq = ctypes.c_double(0.0)
    jmin = lib().pao_table(np.ascontiguousarray(h, np.uint32), n, N, R, R_tilde, float(dbeta),
                           fl, T, tau, ctypes.byref(lnq))
    return fl, T, tau, lnq.value, jmin


def copy_counts(U, fl, T, seed: int, step: int) -> np.ndarray:
    n = np.zeros(U.size, np.uint32)
    lib().pao_copy_counts(np.ascontiguousarray(U, np.int32), U.size, fl, T, seed, step, n)
    return n


def culling_fraction(h, R: int, dbeta: float) -> float:
    return lib().pao_culling_fraction(np.ascontiguousarray(h, np.uint32), h.size, R, float(dbeta))


def choose_dbeta(h, R: int, eps_target: float, rem: float):
    """Constant-culling step: returns (dbeta, reached_end) or raises."""
    d = ctypes.c_double(0.0)
    e = ctypes.c_int(0)
    rc = lib().pao_choose_dbeta(np.ascontiguousarray(h, np.uint32), h.size, R, float(eps_target),
                                float(rem), ctypes.byref(d), ctypes.byref(e))
    if rc != 0:
        raise ValueError("culling fraction already exceeds the target at dbeta = 0")
    return d.value, bool(e.value)


def sum_eta2(fam: np.ndarray, R: int) -> int:
    return int(lib().pao_sum_eta2(np.ascontiguousarray(fam, np.uint32), fam.size, R))


def family_sizes(fam: np.ndarray, R: int, max_eta: int) -> np.ndarray:
    out = np.zeros(max_eta, np.uint64)
    lib().pao_family_sizes(np.ascontiguousarray(fam, np.uint32), fam.size, R, max_eta, out)
    return out


def overlap_hist(N: int, spins_a: np.ndarray, spins_b: np.ndarray):
    Ra = spins_a.size // N
    Rb = spins_b.size // N
    hist = np.zeros(65, np.uint64)
    d = np.zeros(min(Ra, Rb), np.uint32)
    lib().pao_overlap_hist(N, np.ascontiguousarray(spins_a, np.int8), Ra,
                           np.ascontiguousarray(spins_b, np.int8), Rb, hist, d)
    return hist, d


def link_overlap(L: int, spins_a: np.ndarray, spins_b: np.ndarray):
    """Link overlap of replica i of a with replica i of b (Sec. II.A): D[i]
    bonds with s^a_n s^a_m s^b_n s^b_m = -1, q_l = 1 - 2 D / (3N), and the
    counts of D = 0..3N."""
    N = L ** 3
    n = min(spins_a.size // N, spins_b.size // N)
    D = np.zeros(n, np.uint32)
    lib().pao_link_overlap(L, np.ascontiguousarray(spins_a, np.int8), spins_a.size // N,
                           np.ascontiguousarray(spins_b, np.int8), spins_b.size // N, D)
    hist = np.bincount(D, minlength=3 * N + 1).astype(np.uint64)
    return hist, D


def density_of_states(L: int, J: np.ndarray) -> np.ndarray:
    g = np.zeros(3 * L ** 3 + 1, np.uint64)
    rc = lib().pao_density_of_states(L, np.ascontiguousarray(J, np.int8), g)
    if rc != 0:
        raise ValueError("lattice too large to enumerate")
    return g


# ---------------------------------------------------------------------------
# the annealing loop (Sec. II)
# ---------------------------------------------------------------------------
@dataclass
class StepRecord:
    k: int
    beta: float
    dbeta: float
    lnQ: float
    beta_F: float
    mean_E: float
    rho_t: float
    R_tilde: int
    E_min: int
    eps_expected: float
    n_culled: int
    sum_eta2: int
    n_at_E_min: int = 0   # replicas at the lowest energy (ground-state estimators, Sec. II.A)


def default_capacity(R: int) -> int:
    return int(R + 16 * math.isqrt(R) + 256)


class Population:
    """One PA population: spins [slot][site] int8, U, family labels.

    ``seed`` keys every draw of this population (init, sweeps, resampling).
    ``t`` is the population's sweep counter, ``k`` its resampling-step index.
    """

    def __init__(self, L: int, J: np.ndarray, R: int, seed: int, capacity: int | None = None):
        self.L = L
        self.N = L ** 3
        self.n_levels = 3 * self.N + 1
        self.J = np.ascontiguousarray(J, np.int8)
        assert self.J.size == 3 * self.N
        self.R = int(R)
        self.seed = int(seed)
        self.capacity = int(capacity) if capacity else default_capacity(R)
        self.spins = np.zeros(self.R * self.N, np.int8)
        self.U = np.zeros(self.R, np.int32)
        self.fam = np.zeros(self.R, np.uint32)
        lib().pao_init(L, self.J, self.R, self.seed, self.spins, self.U, self.fam)
        self.R_tilde = self.R
        self.t = 0
        self.k = 0
        self.beta = 0.0
        self.sum_lnQ = 0.0
        self.last = None  # details of the last resampling step

    # -- C-10: Metropolis sweeps ------------------------------------------
    def sweep(self, beta: float, n_sweeps: int):
        thr = thresholds(beta)
        lib().pao_sweep(self.L, self.J, self.spins, self.U, self.R_tilde, self.seed, thr,
                        self.t, int(n_sweeps))
        self.t += int(n_sweeps)

    def histogram(self) -> np.ndarray:
        return histogram(self.U[: self.R_tilde], self.n_levels)

    # -- C-7 / C-8: resampling beta -> beta_next --------------------------
    def resample(self, beta_next: float):
        dbeta = beta_next - self.beta
        h = self.histogram()
        fl, T, tau, lnQ, jmin = table(h, self.N, self.R, self.R_tilde, dbeta)
        step = self.k + 1
        n = copy_counts(self.U[: self.R_tilde], fl, T, self.seed, step)
        new_spins = np.zeros(self.capacity * self.N, np.int8)
        new_U = np.zeros(self.capacity, np.int32)
        new_fam = np.zeros(self.capacity, np.uint32)
        offsets = np.zeros(self.R_tilde, np.uint64)
        Rn = lib().pao_copy_eliminate(self.L, n, self.R_tilde, self.capacity, self.spins, self.U,
                                      self.fam, new_spins, new_U, new_fam, offsets)
        if Rn < 0:
            raise OverflowError("resampled population exceeds capacity")
        eps = culling_fraction(h, self.R, dbeta)
        self.last = dict(h=h, fl=fl, T=T, tau=tau, n=n, offsets=offsets, jmin=jmin, lnQ=lnQ,
                         dbeta=dbeta, eps=eps, n_culled=int(np.count_nonzero(n == 0)))
        self.spins = new_spins[: Rn * self.N].copy()
        self.U = new_U[:Rn].copy()
        self.fam = new_fam[:Rn].copy()
        self.R_tilde = int(Rn)
        self.sum_lnQ = self.sum_lnQ + lnQ
        self.beta = beta_next
        self.k = step

    # -- C-9: constant culling fraction -----------------------------------
    def choose_beta(self, eps_target: float, beta_max: float):
        rem = beta_max - self.beta
        dbeta, end = choose_dbeta(self.histogram(), self.R, eps_target, rem)
        return beta_max if end else self.beta + dbeta

    # -- C-11: observables --------------------------------------------------
    def observables(self) -> StepRecord:
        h = self.histogram()
        N = self.N
        levels = np.arange(self.n_levels, dtype=np.int64)
        sumE = int(np.sum(h.astype(np.int64) * (2 * levels - 3 * N)))
        mean_E = float(sumE) / float(self.R_tilde)
        beta_F = -(float(N) * math.log(2.0) + self.sum_lnQ)
        s2 = sum_eta2(self.fam, self.R)
        rho_t = float(s2) / float(self.R)
        jmin = int(np.flatnonzero(h)[0])
        E_min = 2 * jmin - 3 * N
        last = self.last or {}
        return StepRecord(k=self.k, beta=self.beta, dbeta=last.get("dbeta", 0.0),
                          lnQ=last.get("lnQ", 0.0), beta_F=beta_F, mean_E=mean_E, rho_t=rho_t,
                          R_tilde=self.R_tilde, E_min=E_min, eps_expected=last.get("eps", 0.0),
                          n_culled=last.get("n_culled", 0), sum_eta2=s2,
                          n_at_E_min=int(h[jmin]))

    def spins_2d(self) -> np.ndarray:
        return self.spins.reshape(self.R_tilde, self.N)


def linear_schedule(beta_max: float, n_temps: int):
    """beta_k = (beta_max * k) / (N_T - 1), k = 0..N_T-1 (FP64, not accumulated)."""
    return [(beta_max * k) / (n_temps - 1) for k in range(n_temps)]


def run_linear(L, J, R, seed, beta_max, n_temps, n_sweeps, capacity=None, partner_seed=None,
               on_step=None):
    """Fixed linear schedule.  With ``partner_seed`` a second population with
    the same couplings runs in lockstep and the overlap histogram is recorded."""
    pops = [Population(L, J, R, seed, capacity)]
    if partner_seed is not None:
        pops.append(Population(L, J, R, partner_seed, capacity))
    betas = linear_schedule(beta_max, n_temps)
    records = []
    for k in range(1, n_temps):
        recs = []
        for p in pops:
            p.resample(betas[k])
            p.sweep(betas[k], n_sweeps)
            recs.append(p.observables())
        q = None
        if len(pops) == 2:
            q, _ = overlap_hist(pops[0].N, pops[0].spins, pops[1].spins)
        records.append((recs, q))
        if on_step is not None:
            on_step(k, pops)
    return pops, records


def run_adaptive(L, J, R, seed, eps_target, beta_max, n_sweeps, capacity=None, max_steps=100000,
                 on_step=None):
    """Constant-culling schedule: each step's dbeta from choose_beta."""
    p = Population(L, J, R, seed, capacity)
    records = []
    while p.beta < beta_max and p.k < max_steps:
        b = p.choose_beta(eps_target, beta_max)
        p.resample(b)
        p.sweep(b, n_sweeps)
        records.append(p.observables())
        if on_step is not None:
            on_step(p.k, p)
    return p, records


# ---------------------------------------------------------------------------
# Gaussian couplings (Sec. II.A), quantised: J = k / 16, k in [-127, 127];
# energies in quanta of 1/16 (E16).  Same loop, draws and copy rule as above;
# the energy levels of the resampling table are the occupied window of E16.
# ---------------------------------------------------------------------------
G_UNIT = 1.0 / 16.0


def g_energy(L: int, K: np.ndarray, spins: np.ndarray) -> np.ndarray:
    spins = np.ascontiguousarray(spins, np.int8)
    R = spins.size // L ** 3
    E = np.zeros(R, np.int32)
    lib().pao_g_energy(L, np.ascontiguousarray(K, np.int8), spins, R, E)
    return E


def g_dE_max(L: int, K: np.ndarray) -> int:
    """Largest |dE16| of a single flip: 2 max over sites of sum_j |k_ij|."""
    N = L ** 3
    nb = np.zeros(N * 6, np.int32)
    bd = np.zeros(N * 6, np.int32)
    lib().pao_neighbours(L, nb, bd)
    k = np.abs(np.asarray(K, np.int64))[bd].reshape(N, 6).sum(axis=1)
    return int(2 * k.max())


def g_thresholds(beta: float, dEmax: int) -> np.ndarray:
    out = np.zeros(dEmax + 1, np.uint64)
    lib().pao_g_thresholds(float(beta), int(dEmax), out)
    return out


def g_sweep_slots(L: int, K: np.ndarray, spins: np.ndarray, E16: np.ndarray, slots: np.ndarray,
                  seed: int, beta: float, t0: int, n_sweeps: int):
    """Sweep selected replicas in place; row i sits in population slot slots[i]."""
    assert spins.dtype == np.int8 and spins.flags.c_contiguous
    assert E16.dtype == np.int32 and E16.flags.c_contiguous
    slots = np.ascontiguousarray(slots, np.uint32)
    lib().pao_g_sweep_slots(L, np.ascontiguousarray(K, np.int8), spins.reshape(-1), E16,
                            slots.size, slots, seed, g_thresholds(beta, g_dE_max(L, K)), t0,
                            n_sweeps)


def g_density_of_states(L: int, K: np.ndarray):
    """(g, off): g[E16 + off] = number of states with energy E16 / 16."""
    off = 3 * 127 * L ** 3
    g = np.zeros(2 * off + 1, np.uint64)
    if lib().pao_g_density_of_states(L, np.ascontiguousarray(K, np.int8), g) != 0:
        raise ValueError("lattice too large to enumerate")
    return g, off


class GaussPopulation(Population):
    """A PA population with quantised Gaussian couplings K (J = K / 16).

    ``U`` holds E16, the energy in quanta of 1/16; the resampling levels are
    the occupied window [min E16, max E16]."""

    def __init__(self, L: int, K: np.ndarray, R: int, seed: int, capacity: int | None = None):
        super().__init__(L, K, R, seed, capacity)     # spins and labels as for +-J
        self.U = g_energy(L, self.J, self.spins)
        self.dEmax = g_dE_max(L, self.J)

    def sweep(self, beta: float, n_sweeps: int):
        slots = np.arange(self.R_tilde, dtype=np.uint32)
        lib().pao_g_sweep_slots(self.L, self.J, self.spins, self.U, self.R_tilde, slots,
                                self.seed, g_thresholds(beta, self.dEmax), self.t, int(n_sweeps))
        self.t += int(n_sweeps)

    def window(self):
        E = self.U[: self.R_tilde]
        return int(E.min()), int(E.max())

    def histogram(self) -> np.ndarray:
        lo, hi = self.window()
        return histogram(self.U[: self.R_tilde] - lo, hi - lo + 1)

    def resample(self, beta_next: float):
        dbeta = beta_next - self.beta
        lo, hi = self.window()
        h = self.histogram()
        n = h.size
        fl = np.zeros(n, np.uint32)
        T = np.zeros(n, np.uint64)
        tau = np.zeros(n, np.float64)
        lnq = ctypes.c_double(0.0)
        jmin = lib().pao_table_unit(h, n, G_UNIT, lo, self.R, self.R_tilde, float(dbeta), fl, T,
                                    tau, ctypes.byref(lnq))
        step = self.k + 1
        level = np.ascontiguousarray(self.U[: self.R_tilde] - lo, np.int32)
        cnt = copy_counts(level, fl, T, self.seed, step)
        new_spins = np.zeros(self.capacity * self.N, np.int8)
        new_U = np.zeros(self.capacity, np.int32)
        new_fam = np.zeros(self.capacity, np.uint32)
        offsets = np.zeros(self.R_tilde, np.uint64)
        Rn = lib().pao_copy_eliminate(self.L, cnt, self.R_tilde, self.capacity, self.spins, self.U,
                                      self.fam, new_spins, new_U, new_fam, offsets)
        if Rn < 0:
            raise OverflowError("resampled population exceeds capacity")
        eps = lib().pao_culling_fraction_unit(h, n, G_UNIT, self.R, float(dbeta))
        self.last = dict(h=h, fl=fl, T=T, tau=tau, n=cnt, offsets=offsets, jmin=jmin,
                         lnQ=lnq.value, dbeta=dbeta, eps=eps, E_lo=lo,
                         n_culled=int(np.count_nonzero(cnt == 0)))
        self.spins = new_spins[: Rn * self.N].copy()
        self.U = new_U[:Rn].copy()
        self.fam = new_fam[:Rn].copy()
        self.R_tilde = int(Rn)
        self.sum_lnQ = self.sum_lnQ + lnq.value
        self.beta = beta_next
        self.k = step

    def choose_beta(self, eps_target: float, beta_max: float):
        rem = beta_max - self.beta
        h = self.histogram()
        d = ctypes.c_double(0.0)
        e = ctypes.c_int(0)
        rc = lib().pao_choose_dbeta_unit(h, h.size, G_UNIT, self.R, float(eps_target), float(rem),
                                         ctypes.byref(d), ctypes.byref(e))
        if rc != 0:
            raise ValueError("culling fraction already exceeds the target at dbeta = 0")
        return beta_max if e.value else self.beta + d.value

    def observables(self) -> StepRecord:
        """As Population.observables; E_min is in quanta (E16), mean_E in units of J."""
        E = self.U[: self.R_tilde].astype(np.int64)
        sumE = int(E.sum())
        mean_E = float(sumE) / float(self.R_tilde) * G_UNIT
        beta_F = -(float(self.N) * math.log(2.0) + self.sum_lnQ)
        s2 = sum_eta2(self.fam, self.R)
        E_min = int(E.min())
        last = self.last or {}
        return StepRecord(k=self.k, beta=self.beta, dbeta=last.get("dbeta", 0.0),
                          lnQ=last.get("lnQ", 0.0), beta_F=beta_F, mean_E=mean_E,
                          rho_t=float(s2) / float(self.R), R_tilde=self.R_tilde, E_min=E_min,
                          eps_expected=last.get("eps", 0.0), n_culled=last.get("n_culled", 0),
                          sum_eta2=s2, n_at_E_min=int(np.count_nonzero(E == E_min)))


# ---------------------------------------------------------------------------
# Gaussian couplings, continuous (Sec. II.A): J on the grid 2^-32, |J| < 8, so
# every energy is exact in FP64.  Same loop, draws and copy rule as above; the
# resampling works on per-replica weights instead of energy levels (there are
# no levels to group by), with the normaliser S of Eq. 2 and the culled mass
# of Sec. III.C summed in fixed point (pa_oracle.c, pao_r_fixsum96).
# ---------------------------------------------------------------------------
R_GRID = 2.0 ** -32


def r_exp(x) -> np.ndarray:
    """pao_r_exp elementwise (exp for x <= 0 by a fixed IEEE sequence)."""
    x = np.ascontiguousarray(np.atleast_1d(x), np.float64)
    out = np.zeros_like(x)
    lib().pao_r_exp_many(x, x.size, out)
    return out


def r_energy(L: int, J: np.ndarray, spins: np.ndarray) -> np.ndarray:
    spins = np.ascontiguousarray(spins, np.int8)
    R = spins.size // L ** 3
    E = np.zeros(R, np.float64)
    lib().pao_r_energy(L, np.ascontiguousarray(J, np.float64), spins, R, E)
    return E


def r_fixsum96(v: np.ndarray) -> int:
    """sum_i floor(v_i 2^96) for v_i in [0, 1], as an exact Python int."""
    v = np.ascontiguousarray(v, np.float64)
    out = np.zeros(2, np.uint64)
    lib().pao_r_fixsum96(v, v.size, out)
    return (int(out[1]) << 64) | int(out[0])


def r_round96(total: int) -> float:
    """A fixed-point sum rounded once to FP64 (nearest, ties to even) and
    scaled by 2^-96 (exact)."""
    return math.ldexp(float(total), -96)


def r_weights(E: np.ndarray, dbeta: float, E_min: float) -> np.ndarray:
    E = np.ascontiguousarray(E, np.float64)
    w = np.zeros_like(E)
    lib().pao_r_weights(E, E.size, float(dbeta), float(E_min), w)
    return w


def r_normaliser(w: np.ndarray) -> float:
    """S = sum of the weights (Eq. 2 up to the factor 1/R~), fixed point."""
    return r_round96(r_fixsum96(w))


def r_culling_fraction(E: np.ndarray, R: int, dbeta: float) -> float:
    """eps(dbeta) = (sum over replicas with tau < 1 of (1 - tau)) / R."""
    E = np.ascontiguousarray(E, np.float64)
    w = r_weights(E, dbeta, float(E.min()))
    S = r_normaliser(w)
    c = np.zeros_like(w)
    lib().pao_r_cull_terms(w, w.size, int(R), S, c)
    return r_round96(r_fixsum96(c)) / float(R)


def r_choose_dbeta(E: np.ndarray, R: int, eps_target: float, rem: float):
    """The constant-culling bisection of pao_choose_dbeta_unit (Sec. III.C),
    with r_culling_fraction: (dbeta, reached_end) or ValueError."""
    if r_culling_fraction(E, R, 0.0) > eps_target:
        raise ValueError("culling fraction already exceeds the target at dbeta = 0")
    if r_culling_fraction(E, R, rem) <= eps_target:
        return rem, True
    lo, hi = 0.0, rem
    for _ in range(64):
        mid = lo + 0.5 * (hi - lo)
        if r_culling_fraction(E, R, mid) <= eps_target:
            lo = mid
        else:
            hi = mid
    return lo, False


def r_exact_thermo(L: int, J: np.ndarray, betas):
    """(lnZ, <E>, var E, E0) per beta by enumerating all 2^N states (N <= 30)."""
    betas = np.ascontiguousarray(betas, np.float64)
    n = betas.size
    lnZ, Em, vE = np.zeros(n), np.zeros(n), np.zeros(n)
    E0 = ctypes.c_double(0.0)
    if lib().pao_r_exact_thermo(L, np.ascontiguousarray(J, np.float64), n, betas, lnZ, Em, vE,
                                ctypes.byref(E0)) != 0:
        raise ValueError("lattice too large to enumerate")
    return lnZ, Em, vE, E0.value


class GaussRealPopulation(Population):
    """A PA population with real Gaussian couplings J (FP64 on the 2^-32 grid).

    ``U`` holds the energies (FP64, exact).  Initial spins and family labels
    are those of every model (Philox INIT draws)."""

    def __init__(self, L: int, J: np.ndarray, R: int, seed: int, capacity: int | None = None):
        super().__init__(L, np.ones(3 * L ** 3, np.int8), R, seed, capacity)
        J = np.ascontiguousarray(J, np.float64)
        assert J.size == 3 * self.N
        assert np.all(np.abs(J) < 8.0) and np.all(np.ldexp(J, 32) == np.rint(np.ldexp(J, 32)))
        self.J = J
        self.U = r_energy(L, J, self.spins)

    def sweep(self, beta: float, n_sweeps: int):
        slots = np.arange(self.R_tilde, dtype=np.uint32)
        lib().pao_r_sweep_slots(self.L, self.J, self.spins, self.U, self.R_tilde, slots,
                                self.seed, float(beta), self.t, int(n_sweeps))
        self.t += int(n_sweeps)

    def histogram(self):
        raise TypeError("continuous energies have no level histogram")

    def resample(self, beta_next: float):
        dbeta = beta_next - self.beta
        E = self.U[: self.R_tilde]
        E_min = float(E.min())
        w = r_weights(E, dbeta, E_min)
        S = r_normaliser(w)
        step = self.k + 1
        cnt = np.zeros(self.R_tilde, np.uint32)
        tau = np.zeros(self.R_tilde, np.float64)
        lib().pao_r_copy_counts(w, self.R_tilde, self.R, S, self.seed, step, cnt, tau)
        total = int(cnt.astype(np.uint64).sum())
        offsets = np.zeros(self.R_tilde, np.uint64)
        offsets[1:] = np.cumsum(cnt[:-1].astype(np.uint64))
        if total > self.capacity:
            raise OverflowError("resampled population exceeds capacity")
        # copy / eliminate (Sec. II): copies of replica i fill consecutive new
        # slots from offset_i on, in the old order, with i's family label
        src = np.repeat(np.arange(self.R_tilde), cnt.astype(np.int64))
        lnQ = math.log(S) - math.log(float(self.R_tilde)) - dbeta * E_min
        eps = r_culling_fraction(E, self.R, dbeta)
        self.last = dict(w=w, S=S, tau=tau, n=cnt, offsets=offsets, lnQ=lnQ, dbeta=dbeta,
                         eps=eps, E_ref=E_min, n_culled=int(np.count_nonzero(cnt == 0)))
        self.spins = self.spins.reshape(self.R_tilde, self.N)[src].reshape(-1).copy()
        self.U = E[src].copy()
        self.fam = self.fam[: self.R_tilde][src].copy()
        self.R_tilde = total
        self.sum_lnQ = self.sum_lnQ + lnQ
        self.beta = beta_next
        self.k = step

    def choose_beta(self, eps_target: float, beta_max: float):
        rem = beta_max - self.beta
        dbeta, end = r_choose_dbeta(self.U[: self.R_tilde], self.R, eps_target, rem)
        return beta_max if end else self.beta + dbeta

    def observables(self) -> StepRecord:
        """As Population.observables, with E_min an FP64 energy and <E> the
        exact sum of the energies (integers in units 2^-32) rounded once to
        FP64, divided by R~ and scaled by 2^-32."""
        E = self.U[: self.R_tilde]
        q = np.ldexp(E, 32).astype(np.int64)        # exact: |E 2^32| < 2^49
        sumE = (int((q >> 24).sum()) << 24) + int((q & ((1 << 24) - 1)).sum())
        mean_E = float(sumE) / float(self.R_tilde) * R_GRID
        beta_F = -(float(self.N) * math.log(2.0) + self.sum_lnQ)
        s2 = sum_eta2(self.fam, self.R)
        E_min = float(E.min())
        last = self.last or {}
        return StepRecord(k=self.k, beta=self.beta, dbeta=last.get("dbeta", 0.0),
                          lnQ=last.get("lnQ", 0.0), beta_F=beta_F, mean_E=mean_E,
                          rho_t=float(s2) / float(self.R), R_tilde=self.R_tilde, E_min=E_min,
                          eps_expected=last.get("eps", 0.0), n_culled=last.get("n_culled", 0),
                          sum_eta2=s2, n_at_E_min=int(np.count_nonzero(E == E_min)))
