"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the annealing method: it only draws the
disorder (the +-J couplings) and names the seeds and sizes of the workloads.
Every random number the method itself uses comes from the population seed
through the counter-based generator that each implementation carries.

Couplings follow the +-J reading of the Edwards-Anderson model of Sec. II.A
(the paper draws Gaussian J; the integer-energy hot path uses J = +-1 with
probability 1/2 each).  Layout: J[d * N + site] is the bond from ``site`` to
``site + e_d``, d = 0, 1, 2 for x, y, z, site = x + L (y + L z).
"""
from __future__ import annotations

import numpy as np


def couplings_pm(L: int, coupling_seed: int) -> np.ndarray:
    """3 L^3 i.i.d. couplings, +1 or -1 with probability 1/2 (numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(int(coupling_seed)))
    bits = rng.integers(0, 2, size=3 * L ** 3, dtype=np.int8)
    return (1 - 2 * bits).astype(np.int8)


def couplings_gauss16(L: int, coupling_seed: int) -> np.ndarray:
    """3 L^3 Gaussian couplings J ~ N(0, 1) (numpy PCG64) rounded to multiples of
    1/16 and returned as the integers k = 16 J, clipped to [-127, 127]."""
    rng = np.random.Generator(np.random.PCG64(int(coupling_seed)))
    z = rng.standard_normal(3 * L ** 3)
    return np.clip(np.rint(16.0 * z), -127, 127).astype(np.int8)


def couplings_gauss(L: int, coupling_seed: int) -> np.ndarray:
    """3 L^3 Gaussian couplings J ~ N(0, 1) (numpy PCG64) as FP64 numbers rounded
    to the nearest multiple of 2^-32 (ties to even) and kept inside (-8, 8)."""
    rng = np.random.Generator(np.random.PCG64(int(coupling_seed)))
    z = rng.standard_normal(3 * L ** 3)
    k = np.clip(np.rint(np.ldexp(z, 32)), -(2.0 ** 35) + 1, 2.0 ** 35 - 1)
    return np.ldexp(k, -32)


def couplings_ferro(L: int) -> np.ndarray:
    """All couplings +1 (the ferromagnetic limit)."""
    return np.ones(3 * L ** 3, np.int8)


def population_seed(config: int, instance: int, pop: int) -> int:
    """Population seed for (workload config, instance, population)."""
    return 0x5EED0000 + (config << 16) + instance * 2 + pop


def coupling_seed(config: int, instance: int) -> int:
    return 0xC0DE0000 + (config << 16) + instance


# Workloads (sizes of the paper's kind of run: L, R, schedule, sweeps).
WORKLOADS = {
    "c1_l4": dict(L=4, R=1000, n_temps=51, beta_max=5.0, n_sweeps=10, layout="int8", pops=1),
    "c2_l8": dict(L=8, R=100000, n_temps=201, beta_max=5.0, n_sweeps=10, layout="int8", pops=2),
    "c3_l10": dict(L=10, R=500000, eps=0.1, beta_max=5.0, n_sweeps=10, layout="bitpack64",
                   pops=1),
}


def serving_requests(duration_s: float = 600.0, rate: float = 4.0, seed: int = 0x5E4E,
                     Ls=(4, 6, 8, 10, 12), R_lo: float = 1e4, R_hi: float = 2e5,
                     n_temps_lo: int = 51, n_temps_hi: int = 201):
    """A Poisson stream of PA requests (numpy PCG64): exponential inter-arrival
    times of mean 1/rate up to duration_s; L uniform over Ls; R log-uniform on
    [R_lo, R_hi]; n_temps uniform on [n_temps_lo, n_temps_hi].  Request i uses
    coupling_seed(5, i) and population_seed(5, i, 0)."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    out = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration_s:
            break
        i = len(out)
        out.append(dict(rid=i, arrival=t, L=int(rng.choice(Ls)),
                        R=int(round(float(np.exp(rng.uniform(np.log(R_lo), np.log(R_hi)))))),
                        n_temps=int(rng.integers(n_temps_lo, n_temps_hi + 1)),
                        coupling_seed=coupling_seed(5, i), seed=population_seed(5, i, 0)))
    return out
