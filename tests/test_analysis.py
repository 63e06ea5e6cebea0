"""Estimators over PA runs (CPU): rho_f from independent runs against the
paper's family-statistic relation, and the ground-state estimators against
exact enumeration.  The runs here are the oracle's; the estimators are the
package's host-side arithmetic (paper_1711_02146_amd.analysis), which the GPU
drivers feed with the library's per-step records.

Amey & Machta, arXiv:1711.02146: Sec. III.A (rho_f, rho_t), Sec. III.E
(rho_t - 1 = 2 eps k, rho_f = 2 pi eps^2 k in the MCMC-equilibrated regime),
Sec. V.A (error of a sample variance), Sec. II.A (ground-state estimators).
"""
import json
import math
import os

import numpy as np

import oracle
import pa_inputs
from paper_1711_02146_amd import analysis

HERE = os.path.dirname(os.path.abspath(__file__))


def test_rho_f_estimate_definition():
    x = np.array([[1.0, 2.0], [3.0, 2.0], [5.0, 2.0]])
    rf, drf = analysis.rho_f_estimate(x, 100)
    np.testing.assert_allclose(rf, [100 * 4.0, 0.0])
    np.testing.assert_allclose(drf, [math.sqrt(2 / 2) * 400.0, 0.0])


def test_rho_f_predicted_constant_eps():
    eps = np.full(7, 0.1)
    rho_t = 1 + 2 * 0.1 * np.arange(1, 8)
    pred = analysis.rho_f_predicted(rho_t, eps)
    # rho_t - 1 = 2 eps k  =>  prediction = 2 pi eps^2 k
    np.testing.assert_allclose(pred, 2 * math.pi * 0.01 * np.arange(1, 8))


def test_paper_sweep_schedule():
    assert [analysis.paper_sweep_schedule(b) for b in (0.0, 0.49, 0.5, 2.5, 2.51, 5.0)] == \
        [3, 3, 22, 22, 1, 1]


def test_rho_f_relation_high_temperature():
    """M = 48 independent oracle runs of one L = 4 instance on a constant-culling
    schedule (eps = 0.1, recorded once and reused): rho_f = R var(beta F~)
    agrees with rho_t - 1 - sum (2 eps - 2 pi eps^2) within its error, and
    rho_t - 1 >= rho_f."""
    L, R, K, M = 4, 3000, 16, 48
    J = pa_inputs.couplings_pm(L, 4242)
    p = oracle.Population(L, J, R, 99)
    betas = [0.0]
    for _ in range(K):
        b = p.choose_beta(0.1, 5.0)
        p.resample(b)
        p.sweep(b, 10)
        betas.append(b)
    bF = np.zeros((M, K))
    rt = np.zeros((M, K))
    eps = np.zeros((M, K))
    for m in range(M):
        q = oracle.Population(L, J, R, 777 + m)
        for k in range(1, K + 1):
            q.resample(betas[k])
            q.sweep(betas[k], 10)
            o = q.observables()
            bF[m, k - 1], rt[m, k - 1], eps[m, k - 1] = o.beta_F, o.rho_t, o.eps_expected
    rf, drf = analysis.rho_f_estimate(bF, R)
    pred = analysis.rho_f_predicted(rt.mean(axis=0), eps.mean(axis=0))
    k = K - 1
    assert abs(eps.mean() - 0.1) < 0.01
    assert abs(rf[k] - pred[k]) < 3 * drf[k], (rf[k], drf[k], pred[k])
    assert rf[k] <= rt.mean(axis=0)[k] - 1
    # the MCMC-equilibrated form: rho_t - 1 = 2 eps k within 5%
    assert abs((rt.mean(axis=0)[k] - 1) / (2 * eps.mean(axis=0).sum()) - 1) < 0.05


def test_ground_state_estimators_l3_exact():
    """PA at L = 3 (oracle) to beta = 5: the fraction at the lowest energy found
    (g0~) and the Boltzmann estimate d exp(-beta E0 + beta F~) (d = number of
    ground states) against exact enumeration."""
    gold = json.load(open(os.path.join(HERE, "golden", "l3_exact.json")))
    L, N = 3, 27
    J = pa_inputs.couplings_pm(L, gold["coupling_seed"])
    g = np.array(gold["dos"], dtype=np.float64)
    U0 = int(np.flatnonzero(g)[0])
    E0_exact = 2 * U0 - 3 * N
    R = 20000
    betas = oracle.linear_schedule(5.0, 51)
    p = oracle.Population(L, J, R, 31337)
    E_min, n0, Rt, bF = [], [], [], []
    for k in range(1, len(betas)):
        p.resample(betas[k])
        p.sweep(betas[k], 10)
        o = p.observables()
        E_min.append(o.E_min)
        n0.append(o.n_at_E_min)
        Rt.append(o.R_tilde)
        bF.append(o.beta_F)
    E0, g_tilde, g_bar = analysis.ground_state_estimates(E_min, n0, Rt, betas[1:], bF,
                                                         degeneracy=int(g[U0]))
    assert E0 == E0_exact
    U = np.arange(g.size)
    for k in (24, 49):          # beta = 2.5 and 5
        b = betas[k + 1]
        w = g * np.exp(-b * (2 * U - 3 * N) - (-b * E0_exact))
        g0 = g[U0] / w.sum()
        rho_t = p.observables().rho_t
        err = math.sqrt(g0 * (1 - g0) * max(rho_t, 1.0) / R) + 1e-3
        assert abs(g_tilde[k] - g0) < 5 * err, (b, g_tilde[k], g0)
        assert abs(g_bar[k] - g0) < 5 * err + 0.02 * g0, (b, g_bar[k], g0)


def test_link_overlap_mean_and_katzgraber_young_arithmetic():
    """<q_l> from a D histogram (q_l = 1 - 2 D / 3N) and e_l = -beta sigma^2 3 (1 - <q_l>)
    (Sec. II.A), on histograms whose answer is known."""
    N = 4 ** 3
    h = np.zeros(3 * N + 1, np.uint64)
    h[0] = 5
    assert analysis.link_overlap_mean(h, N) == 1.0
    h[:] = 0
    h[3 * N] = 2
    assert analysis.link_overlap_mean(h, N) == -1.0
    h[:] = 0
    h[3 * N // 2] = 7  # half the bonds differ: q_l = 0
    assert analysis.link_overlap_mean(h, N) == 0.0
    e_l, d = analysis.katzgraber_young(0.5, -1.25, 0.0)
    assert e_l == -1.5 and d == -0.25
    e_l, _ = analysis.katzgraber_young(2.0, 0.0, 1.0, coupling_variance=1.3)
    assert e_l == 0.0


def test_quantised_gauss_variance_is_sheppard():
    """Rounding a unit normal to multiples of h adds h^2 / 12 to its variance
    (Sheppard's correction; the remainder is of order exp(-2 pi^2 / h^2))."""
    assert abs(analysis.quantised_gauss_variance() - (1.0 + 1.0 / (12 * 256))) < 1e-12
    assert abs(analysis.quantised_gauss_variance(1.0, 40) - (1.0 + 1.0 / 12)) < 1e-6
