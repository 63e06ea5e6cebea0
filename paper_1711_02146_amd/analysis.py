"""Estimators and drivers over PA runs on the GPU (Amey & Machta, arXiv:1711.02146).

  * rho_f from M independent runs of one instance (Sec. III.A definition,
    rho_f = R var(beta F~); error of a sample variance, Sec. V.A), and the
    prediction from the family statistic, rho_t - 1 - sum_l (2 eps_l - 2 pi eps_l^2)
    (Sec. III.E; for a constant culling fraction eps the sum is
    (2 eps - 2 pi eps^2) k).
  * A constant-culling beta schedule recorded from one adaptive run and reused
    for other runs (Sec. IV.B), and the paper's sweep schedule (3 sweeps below
    beta = 0.5, 22 up to 2.5, 1 above).
  * Hardness-dependent population size (Sec. IV.A): rerun with R = 150 rho_t
    until R >= 100 rho_t.
  * Ground-state estimators (Sec. II.A): E0~, the lowest energy met during the
    run; g0~(beta), the fraction of the population at E0~; and the Boltzmann
    estimate g0_bar = d exp(-beta E0~ + beta F~) with d the ground-state
    degeneracy (2 for continuous couplings).
  * The link overlap q_l and the Katzgraber-Young equilibration measure
    (Sec. II.A): <q_l> over the pairs of two independent populations,
    e_l = -beta (N_b / N) (1 - <q_l>), and e_l - e, whose average over Gaussian
    disorder samples, Delta_KY, vanishes in equilibrium.

Every step runs in the library's kernels; this module only schedules calls and
reduces the per-step scalars they return.
"""
from __future__ import annotations

import math

import numpy as np


# --- estimators (plain arithmetic on per-run scalars) --------------------------
def rho_f_estimate(beta_F_runs, R: int):
    """rho_f = R var(beta F~) over M independent runs (sample variance), and its
    standard error sqrt(2 / (M - 1)) rho_f for normally distributed beta F~."""
    x = np.asarray(beta_F_runs, dtype=np.float64)
    M = x.shape[0]
    if M < 2:
        raise ValueError("rho_f needs at least two runs")
    rf = R * x.var(axis=0, ddof=1)
    return rf, math.sqrt(2.0 / (M - 1)) * rf


def rho_f_predicted(rho_t, eps_steps):
    """rho_t - 1 - sum over steps l <= k of (2 eps_l - 2 pi eps_l^2), for every k.

    rho_t: [K] (mean over runs) family statistic after each step; eps_steps:
    [K] culling fraction of each step."""
    e = np.asarray(eps_steps, dtype=np.float64)
    return np.asarray(rho_t, dtype=np.float64) - 1.0 - np.cumsum(2.0 * e - 2.0 * math.pi * e * e)


def ground_state_estimates(E_min_steps, n_at_E_min_steps, R_tilde_steps, betas, beta_F_steps,
                           degeneracy: int = 2):
    """E0~ = lowest energy of the run; per step g0~ = (population at E0~) / R~
    (zero where that step's lowest energy is above E0~) and
    g0_bar = degeneracy exp(-beta E0~ + beta F~)."""
    E = np.asarray(E_min_steps, dtype=np.int64)
    n = np.asarray(n_at_E_min_steps, dtype=np.float64)
    Rt = np.asarray(R_tilde_steps, dtype=np.float64)
    b = np.asarray(betas, dtype=np.float64)
    bF = np.asarray(beta_F_steps, dtype=np.float64)
    E0 = int(E.min())
    g_tilde = np.where(E == E0, n / Rt, 0.0)
    g_bar = degeneracy * np.exp(-b * E0 + bF)
    return E0, g_tilde, g_bar


def link_overlap_mean(hist, N: int) -> float:
    """<q_l> over the pairs of a link-overlap histogram: hist[D] pairs with D
    of the N_b = 3N bonds differing, q_l = 1 - 2 D / N_b."""
    h = np.asarray(hist, dtype=np.float64)
    if h.size != 3 * N + 1 or h.sum() == 0:
        raise ValueError("need a non-empty histogram of 3N + 1 bins")
    D = np.arange(h.size, dtype=np.float64)
    return float(1.0 - 2.0 * (h * D).sum() / (h.sum() * 3 * N))


def katzgraber_young(beta: float, e: float, q_l: float, coupling_variance: float = 1.0):
    """e_l = -beta sigma^2 (N_b / N) (1 - <q_l>) with N_b / N = 3 on the cubic
    lattice, and e_l - e for one disorder sample (e: energy per spin).  The
    paper's form has sigma^2 = 1 (unit-variance Gaussian couplings); the
    relation comes from Gaussian integration by parts, so couplings of
    variance sigma^2 scale it by sigma^2.  Averaged over samples, e_l - e is
    Delta_KY."""
    e_l = -beta * coupling_variance * 3.0 * (1.0 - q_l)
    return e_l, e_l - e


def quantised_gauss_variance(quantum: float = 1.0 / 16.0, kmax: int = 127) -> float:
    """Variance of a unit normal rounded to multiples of `quantum` and clipped
    to +-kmax quanta (the PA_MODEL_GAUSS16 couplings): sum over k of
    (k quantum)^2 times the normal mass of the k-th rounding interval."""
    k = np.arange(-kmax, kmax + 1, dtype=np.float64)
    lo = np.where(k == -kmax, -np.inf, (k - 0.5) * quantum)
    hi = np.where(k == kmax, np.inf, (k + 0.5) * quantum)
    cdf = np.vectorize(lambda x: 0.5 * math.erfc(-x / math.sqrt(2.0)))
    mass = cdf(hi) - cdf(lo)
    return float(((k * quantum) ** 2 * mass).sum())


def paper_sweep_schedule(beta: float) -> int:
    """Sweeps per step of the paper's optimised schedule (Sec. IV.B)."""
    if beta < 0.5:
        return 3
    if beta <= 2.5:
        return 22
    return 1


# --- drivers (GPU) ------------------------------------------------------------
def constant_eps_schedule(L: int, R: int, J, seed: int, eps: float, beta_max: float,
                          n_sweeps=10, layout: str = "bitpack64", max_steps: int = 100000):
    """betas of one constant-culling run (bisection to culling fraction eps,
    Sec. III.C), from beta = 0 to beta_max.  n_sweeps: int or callable(beta)."""
    import paper_1711_02146_amd as pam

    p = pam.Population(L, R, J, seed, layout=layout)
    betas = [0.0]
    try:
        while betas[-1] < beta_max and len(betas) <= max_steps:
            b = p.choose_beta(eps, beta_max)
            p.resample(b)
            p.sweep(b, n_sweeps(b) if callable(n_sweeps) else n_sweeps)
            betas.append(b)
    finally:
        p.close()
    return betas


def replicate_runs(L: int, R: int, J, seeds, betas, n_sweeps=10, layout: str = "bitpack64",
                   capacity: int = 0):
    """M populations of one instance (one per seed) through one schedule, all
    advanced together by a Stepper (one launch set per step).

    n_sweeps: int, a list per step (len(betas) - 1) or callable(beta).
    Returns a dict of [M, K] arrays: beta_F, mean_E, rho_t, eps_expected, E_min,
    n_at_E_min, R_tilde, and the status of every run (0, or the PA status that
    stopped it; its later entries are NaN / -1)."""
    import torch

    import paper_1711_02146_amd as pam

    M, K = len(seeds), len(betas) - 1
    if callable(n_sweeps):
        sweeps = [int(n_sweeps(b)) for b in betas[1:]]
    elif np.ndim(n_sweeps) == 0:
        sweeps = [int(n_sweeps)] * K
    else:
        sweeps = [int(s) for s in n_sweeps]
    if len(sweeps) != K:
        raise ValueError("one sweep count per step")
    stream = torch.cuda.Stream()
    stepper = pam.Stepper(M, L, stream)
    pops = [pam.Population(L, R, J, s, capacity=capacity, layout=layout, stream=stream)
            for s in seeds]
    out = {k: np.full((M, K), np.nan) for k in ("beta_F", "mean_E", "rho_t", "eps_expected")}
    for k in ("E_min", "n_at_E_min", "R_tilde"):
        out[k] = np.full((M, K), -1, dtype=np.int64)
    status = np.zeros(M, dtype=np.int32)
    alive = list(range(M))
    try:
        for k in range(K):
            if not alive:
                break
            obs, st = stepper.step([pops[m] for m in alive], [betas[k + 1]] * len(alive),
                                   [sweeps[k]] * len(alive))
            still = []
            for m, o, s in zip(alive, obs, st):
                if s != 0:
                    status[m] = s
                    continue
                for f in ("beta_F", "mean_E", "rho_t", "eps_expected", "E_min", "n_at_E_min",
                          "R_tilde"):
                    out[f][m, k] = o[f]
                still.append(m)
            alive = still
    finally:
        stepper.close()
        for p in pops:
            p.close()
    out["status"] = status
    out["betas"] = np.asarray(betas, dtype=np.float64)
    out["sweeps"] = np.asarray(sweeps)
    return out


def rho_f_study(runs: dict, R: int):
    """Per step: rho_f +- its error, mean rho_t, mean culling fraction and the
    prediction rho_t - 1 - sum (2 eps - 2 pi eps^2), from replicate_runs output."""
    ok = runs["status"] == 0
    bF = runs["beta_F"][ok]
    rf, drf = rho_f_estimate(bF, R)
    rt = runs["rho_t"][ok].mean(axis=0)
    eps = runs["eps_expected"][ok].mean(axis=0)
    return {"rho_f": rf, "rho_f_err": drf, "rho_t": rt, "eps": eps,
            "rho_f_predicted": rho_f_predicted(rt, eps), "runs": int(ok.sum())}


def link_overlap_run(L: int, J, seeds, betas, n_sweeps=10, model: str = "gauss16",
                     layout: str = "bitpack64", R: int = 2000):
    """Two independent populations of one disorder sample (seeds[0], seeds[1])
    through one schedule; after every step <q_l> between them, e (the two
    populations' mean energy per spin), e_l and e_l - e (Sec. II.A).  J: the
    couplings in the model's form (k = 16 J for "gauss16").  Returns a dict of
    per-step arrays."""
    import paper_1711_02146_amd as pam

    N = L ** 3
    var = quantised_gauss_variance() if model == "gauss16" else 1.0
    pops = [pam.Population(L, R, J, s, layout=layout, model=model) for s in seeds[:2]]
    out = {k: [] for k in ("beta", "q_l", "e", "e_l", "delta")}
    try:
        for k in range(1, len(betas)):
            b = float(betas[k])
            es = []
            for p in pops:
                p.resample(b)
                p.sweep(b, n_sweeps(b) if callable(n_sweeps) else n_sweeps)
                es.append(p.observables()["mean_E"] / N)
            q = link_overlap_mean(pam.link_overlap_hist(pops[0], pops[1]), N)
            e = 0.5 * (es[0] + es[1])
            e_l, d = katzgraber_young(b, e, q, var)
            for key, v in zip(("beta", "q_l", "e", "e_l", "delta"), (b, q, e, e_l, d)):
                out[key].append(v)
    finally:
        for p in pops:
            p.close()
    return {k: np.asarray(v) for k, v in out.items()}


def equilibrate(L: int, J, seed: int, R0: int, betas, n_sweeps=10, layout: str = "bitpack64",
                accept: float = 100.0, grow: float = 150.0, max_rounds: int = 8,
                max_R: int = 1 << 26):
    """Hardness-dependent population size (Sec. IV.A): run with R0; while
    R < accept * rho_t (final), run again with R = ceil(grow * rho_t) and a new
    seed (seed + round).  Returns the list of rounds (R, final observables); the
    last round is the accepted one unless max_rounds or max_R stopped it."""
    rounds = []
    R = int(R0)
    for r in range(max_rounds):
        runs = replicate_runs(L, R, J, [seed + r], betas, n_sweeps, layout)
        if runs["status"][0] != 0:
            rounds.append({"R": R, "status": int(runs["status"][0]), "rho_t": math.nan})
            break
        final = {f: runs[f][0, -1] for f in ("beta_F", "mean_E", "rho_t", "E_min", "R_tilde")}
        rounds.append({"R": R, "status": 0, **final, "accepted": R >= accept * final["rho_t"]})
        if rounds[-1]["accepted"]:
            break
        R_next = int(math.ceil(grow * final["rho_t"]))
        if R_next > max_R:
            break
        R = max(R_next, R + 1)
    return rounds
