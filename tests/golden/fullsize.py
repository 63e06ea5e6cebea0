"""Full-size parity cases and the per-step digests both sides compute.

The two headline workloads, at their real sizes:

  C3  L = 10, R = 5e5, +-J couplings, constant culling eps = 0.1 up to
      beta = 5 (Sec. III.C step choice), N_S = 10: the first C3_STEPS steps
      (the benchmark times a window of this anneal);
  C2  L = 8, R = 1e5, +-J couplings, two populations of the same sample with
      different seeds, linear schedule of 201 temperatures on [0, 5], N_S = 10,
      the 65-bin spin-overlap histogram after every step: the first C2_STEPS.

A digest is SHA-256 of a canonical byte image (spins as one bit per site,
1 <=> s = -1, replicas in slot order, sites in lexicographic order, packed by
numpy.packbits; integer arrays as little-endian 32-bit words).  FP64 scalars
are stored exactly (float.hex).  This module holds no arithmetic of the
method: only the workload constants and the hashing.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

C3 = dict(name="C3", L=10, R=500000, eps=0.1, beta_max=5.0, n_sweeps=10, config=3)
C3_STEPS = 25
C2 = dict(name="C2", L=8, R=100000, beta_max=5.0, n_temps=201, n_sweeps=10, config=2)
C2_STEPS = 10

FLOATS = ("beta", "dbeta", "lnQ", "beta_F", "mean_E", "rho_t", "eps_expected")
INTS = ("R_tilde", "n_culled", "sum_eta2", "E_min", "n_at_E_min")


def path(name: str) -> str:
    return os.path.join(HERE, f"fullsize_{name}.json")


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def spins_digest(spins: np.ndarray, R: int, N: int) -> str:
    """spins: R x N int8 (+1/-1), [replica][site]."""
    s = np.asarray(spins).reshape(R, N)
    return sha(np.packbits(s < 0, axis=1))


def u32_digest(a) -> str:
    return sha(np.asarray(a).astype("<u4"))


def load(name: str) -> dict:
    with open(path(name)) as f:
        return json.load(f)
