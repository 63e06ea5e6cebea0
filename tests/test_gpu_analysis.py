"""GPU: drivers over many runs of one instance (Amey & Machta, arXiv:1711.02146).

  * replicate_runs (M populations of one instance on a Stepper) is bit-exact
    against M oracle runs, with the paper's variable sweep schedule (Sec. IV.B);
  * rho_f from 48 independent GPU runs against rho_t - 1 - sum (2 eps - 2 pi eps^2)
    (Sec. III.E) and rho_t - 1 >= rho_f (Sec. III.B);
  * the hardness-dependent population size loop (Sec. IV.A);
  * ground-state estimators on the ferromagnet (Sec. II.A).
"""
import math

import numpy as np
import pytest

import oracle
import pa_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def an():
    import torch

    assert torch.cuda.is_available()
    import paper_1711_02146_amd as pam
    from paper_1711_02146_amd import analysis

    pam.lib()
    return analysis


def test_replicate_runs_match_oracle(an):
    L, R, M = 6, 700, 3
    J = pa_inputs.couplings_pm(L, 515)
    betas = [0.0, 0.2, 0.45, 0.5, 0.9, 2.5, 2.6, 4.0]
    seeds = [100 + m for m in range(M)]
    runs = an.replicate_runs(L, R, J, seeds, betas, an.paper_sweep_schedule)
    assert list(runs["sweeps"]) == [3, 3, 22, 22, 22, 1, 1]
    assert np.all(runs["status"] == 0)
    for m, s in enumerate(seeds):
        o = oracle.Population(L, J, R, s)
        for k in range(1, len(betas)):
            o.resample(betas[k])
            o.sweep(betas[k], an.paper_sweep_schedule(betas[k]))
            r = o.observables()
            assert runs["beta_F"][m, k - 1] == r.beta_F
            assert runs["mean_E"][m, k - 1] == r.mean_E
            assert runs["rho_t"][m, k - 1] == r.rho_t
            assert runs["eps_expected"][m, k - 1] == r.eps_expected
            assert runs["E_min"][m, k - 1] == r.E_min
            assert runs["n_at_E_min"][m, k - 1] == r.n_at_E_min
            assert runs["R_tilde"][m, k - 1] == r.R_tilde


def test_rho_f_relation_48_runs(an):
    """48 runs of one L = 6 instance, R = 20000, on a constant-culling schedule
    (eps = 0.1) recorded from one run: high-temperature regime."""
    L, R, M = 6, 20000, 48
    J = pa_inputs.couplings_pm(L, 616)
    betas = an.constant_eps_schedule(L, R, J, 9, 0.1, 0.3)
    assert 10 < len(betas) < 200 and betas[-1] == 0.3
    runs = an.replicate_runs(L, R, J, [2000 + m for m in range(M)], betas, 10)
    st = an.rho_f_study(runs, R)
    assert st["runs"] == M
    k = len(betas) - 2
    assert abs(st["rho_f"][k] - st["rho_f_predicted"][k]) < 3 * st["rho_f_err"][k]
    assert st["rho_f"][k] <= st["rho_t"][k] - 1
    assert abs(np.mean(st["eps"][:-1]) - 0.1) < 0.01   # the last step is clipped at beta_max


def test_equilibrate_grows_population(an):
    L = 6
    J = pa_inputs.couplings_pm(L, 717)
    betas = oracle.linear_schedule(3.0, 31)
    rounds = an.equilibrate(L, J, 4000, 64, betas, 10)
    assert len(rounds) >= 2
    for a, b in zip(rounds, rounds[1:]):
        assert not a["accepted"]
        assert b["R"] == max(math.ceil(150 * a["rho_t"]), a["R"] + 1)
    assert rounds[-1]["accepted"] and rounds[-1]["R"] >= 100 * rounds[-1]["rho_t"]


def test_ground_state_ferromagnet(an):
    """All J = +1: E0 = -3N, two ground states.  On a constant-culling schedule
    (eps = 0.1, so the free-energy estimate is equilibrated through the ordering
    transition) almost the whole population sits in them at beta = 5, and
    2 exp(-beta E0 + beta F~) agrees with that fraction."""
    L, R = 4, 20000
    J = pa_inputs.couplings_ferro(L)
    betas = an.constant_eps_schedule(L, R, J, 6, 0.1, 5.0)
    assert betas[-1] == 5.0
    runs = an.replicate_runs(L, R, J, [5], betas, 10)
    E0, g_tilde, g_bar = an.ground_state_estimates(runs["E_min"][0], runs["n_at_E_min"][0],
                                                   runs["R_tilde"][0], betas[1:],
                                                   runs["beta_F"][0], degeneracy=2)
    assert E0 == -3 * L ** 3
    assert g_tilde[-1] > 0.99
    assert abs(g_bar[-1] - g_tilde[-1]) < 0.05


def test_katzgraber_young_vanishes_over_gaussian_disorder(an):
    """Delta_KY = [e_l - e] over Gaussian disorder samples is zero in
    equilibrium (Sec. II.A; Gaussian integration by parts, exact at any L).
    16 samples at L = 6, two populations each, annealed to beta = 1 (above
    the glass transition, where PA equilibrates easily): the sample mean of
    e_l - e must be within four standard errors of zero, while e and e_l
    themselves are far from zero."""
    L, M = 6, 16
    betas = np.linspace(0.0, 1.0, 16)
    deltas, es = [], []
    for m in range(M):
        K = pa_inputs.couplings_gauss16(L, 700 + m)
        r = an.link_overlap_run(L, K, [2 * m + 1, 2 * m + 2], betas, n_sweeps=5, R=1000)
        assert r["q_l"][0] < r["q_l"][-1]
        deltas.append(r["delta"][-1])
        es.append(r["e"][-1])
    d = np.asarray(deltas)
    se = d.std(ddof=1) / math.sqrt(M)
    print("Delta_KY", d.mean(), "+-", se, "e", np.mean(es), flush=True)
    assert abs(d.mean()) < 4 * se + 1e-3
    assert np.mean(es) < -0.8
