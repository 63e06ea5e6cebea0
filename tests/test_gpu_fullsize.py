"""GPU: whole runs at full size (Amey & Machta, arXiv:1711.02146, Sec. II loop).

The oracle cannot follow these runs step by step in seconds, so every step is
checked against properties that hold at any size, and so are the final
populations: sorted family labels, the energy word of sampled replicas
against the energy of their exported spins, and the overlap histogram against
the exported spins of both populations (tests/props.py; no GPU output is fed
to the oracle):
  * L = 10, R = 5e5, bit-packed, constant culling eps = 0.1 to beta = 5 (the
    benchmark workload, all ~300 steps);
  * L = 8, R = 1e5, int8, two populations, 201 linear temperatures to beta = 5,
    with the 65-bin overlap histogram after every step.
"""
import math

import numpy as np
import pytest

import oracle
import props
import pa_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pam():
    import torch

    assert torch.cuda.is_available()
    import paper_1711_02146_amd as m

    m.lib()
    return m


def check_step(o, prev, L, R, capacity):
    N = L ** 3
    assert 0 < o["R_tilde"] <= capacity
    assert o["rho_t"] >= 1.0 - 1e-12
    assert o["sum_eta2"] >= o["R_tilde"]          # sum of eta^2 >= sum of eta = R~
    assert -3 * N <= o["E_min"] <= 3 * N and (o["E_min"] + 3 * N) % 2 == 0
    assert o["E_min"] <= o["mean_E"] + 1e-9
    assert 1 <= o["n_at_E_min"] <= o["R_tilde"]
    assert o["step"] == prev["step"] + 1
    assert o["beta"] > prev["beta"]
    # the population grows by at most the stated fluctuation bound
    assert abs(o["R_tilde"] - R) <= 16 * math.isqrt(R) + 256


def check_final(pam, g, L, J, n_sample, rng):
    s, u, f = g.export_state()
    R_t = s.shape[0]
    assert np.all(np.diff(f.astype(np.int64)) >= 0)          # family labels stay sorted
    idx = np.sort(rng.choice(R_t, size=min(n_sample, R_t), replace=False))
    np.testing.assert_array_equal(u[idx].astype(np.int32), props.unsatisfied_bonds(L, J, s[idx]))
    return s, u, f


def test_c3_full_anneal(pam):
    L, R, eps, bmax = 10, 500000, 0.1, 5.0
    J = pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(3, 0))
    g = pam.Population(L, R, J, pa_inputs.population_seed(3, 0, 0), layout="bitpack64")
    cap = R + 16 * math.isqrt(R) + 256
    prev = g.observables()
    steps = 0
    while prev["beta"] < bmax:
        b = g.choose_beta(eps, bmax)
        g.resample(b)
        g.sweep(b, 10)
        o = g.observables()
        check_step(o, prev, L, R, cap)
        if b < bmax:
            # the bisection keeps eps(lo) <= target; the step taken is
            # (beta + lo) - beta, which differs from lo by rounding
            assert o["eps_expected"] <= eps + 1e-12
        steps += 1
        prev = o
    assert prev["beta"] == bmax and 100 < steps < 2000
    s, u, f = check_final(pam, g, L, J, 512, np.random.default_rng(3))
    # the reported <E> and E_min are those of the exported population
    E = 2 * u.astype(np.int64) - 3 * L ** 3
    assert prev["mean_E"] == E.sum() / E.size and prev["E_min"] == E.min()
    assert prev["n_at_E_min"] == int(np.count_nonzero(E == E.min()))
    g.close()


def test_c2_two_populations_linear(pam):
    L, R, NT = 8, 100000, 201
    N = L ** 3
    J = pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(2, 0))
    a = pam.Population(L, R, J, pa_inputs.population_seed(2, 0, 0), layout="int8")
    b = pam.Population(L, R, J, pa_inputs.population_seed(2, 0, 1), layout="int8")
    cap = R + 16 * math.isqrt(R) + 256
    betas = oracle.linear_schedule(5.0, NT)
    prev = [a.observables(), b.observables()]
    q2 = []
    for k in range(1, NT):
        obs = []
        for p, pr in zip((a, b), prev):
            p.resample(betas[k])
            p.sweep(betas[k], 10)
            o = p.observables()
            check_step(o, pr, L, R, cap)
            assert o["beta"] == betas[k]
            obs.append(o)
        h = pam.overlap_hist(a, b)
        assert int(h.sum()) == min(obs[0]["R_tilde"], obs[1]["R_tilde"])
        q = (np.arange(65) - 32) / 32.0
        q2.append(float((h * q * q).sum() / h.sum()))
        prev = obs
    # q^2 grows from ~1/N at beta = 0 towards order one in the glassy phase
    assert q2[0] < 0.05 and q2[-1] > 0.2
    rng = np.random.default_rng(2)
    sa, _, _ = check_final(pam, a, L, J, 512, rng)
    sb, _, _ = check_final(pam, b, L, J, 512, rng)
    # the last histogram, recomputed from the exported spins
    n = min(sa.shape[0], sb.shape[0])
    np.testing.assert_array_equal(pam.overlap_hist(a, b), props.overlap_hist65(N, sa, sb))
    a.close()
    b.close()
