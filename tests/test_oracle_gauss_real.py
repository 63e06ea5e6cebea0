"""Pins of the oracle's continuous Gaussian-coupling path (CPU).

Couplings are unit normals (Sec. II.A) rounded to the grid 2^-32, so every
energy is exact in FP64.  The oracle is checked against: the C library's exp
(its own exp within one ulp), exact integer sums (its fixed-point sums),
math.fsum (the correctly rounded sum), the +-J and 1/16-quantised models it
must reduce to when the couplings are +-1 or multiples of 1/16 (both pinned on
their own), the Boltzmann law of its Metropolis chain, and whole PA runs at
L = 3 against the exact free energy and energy of two independent exact
routes (enumeration of 2^27 states, layer transfer matrix), per Sec. II,
Eq. 9 and Sec. III.C of Amey & Machta (arXiv:1711.02146)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import pa_inputs
from oracle.exact import TransferMatrixL3

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def gold():
    return json.load(open(os.path.join(HERE, "golden", "l3_gauss_exact.json")))


def test_exp_within_one_ulp_of_the_c_library():
    rng = np.random.default_rng(1)
    x = np.concatenate([-rng.uniform(0, 708, 100000), -rng.uniform(0, 1, 50000),
                        -np.ldexp(rng.uniform(0, 1, 20000), -rng.integers(1, 60, 20000))])
    y = oracle.r_exp(x)
    ref = np.exp(x)
    assert np.all(np.abs(y - ref) <= np.spacing(ref))
    assert np.mean(y == ref) > 0.85
    # special values: exp(0) = 1, exp(-k ln 2) = 2^-k, the underflow cut
    assert oracle.r_exp([0.0, -0.0]).tolist() == [1.0, 1.0]
    for k in (1, 2, 10, 100):
        assert oracle.r_exp(-k * math.log(2.0))[0] == pytest.approx(2.0 ** -k, rel=2e-16)
    assert oracle.r_exp(-708.0)[0] > 0.0
    assert oracle.r_exp([-708.0000001, -745.0, -1e300]).tolist() == [0.0, 0.0, 0.0]


def test_couplings_are_unit_normals_on_the_grid():
    J = pa_inputs.couplings_gauss(10, 3)
    assert J.dtype == np.float64 and J.size == 3000
    assert np.all(np.ldexp(J, 32) == np.rint(np.ldexp(J, 32)))
    assert np.all(np.abs(J) < 8.0)
    assert abs(J.mean()) < 0.06 and abs(J.var() - 1.0) < 0.08


def test_energy_reduces_to_the_pinned_models():
    L = 4
    N = L ** 3
    rng = np.random.default_rng(5)
    s = rng.choice(np.array([-1, 1], np.int8), size=(7, N))
    # +-J couplings as reals: E = 2U - 3N of the +-J oracle
    Jpm = pa_inputs.couplings_pm(L, 12)
    U = oracle.energy(L, Jpm, s.reshape(-1))
    np.testing.assert_array_equal(oracle.r_energy(L, Jpm.astype(np.float64), s.reshape(-1)),
                                  (2 * U - 3 * N).astype(np.float64))
    # J = k/16: E = E16/16 of the quantised oracle
    K = pa_inputs.couplings_gauss16(L, 11)
    E16 = oracle.g_energy(L, K, s.reshape(-1))
    np.testing.assert_array_equal(oracle.r_energy(L, K / 16.0, s.reshape(-1)), E16 / 16.0)
    # real couplings: global flip symmetry, linearity in J, all-up energy
    J = pa_inputs.couplings_gauss(L, 13)
    E = oracle.r_energy(L, J, s.reshape(-1))
    np.testing.assert_array_equal(E, oracle.r_energy(L, J, (-s).reshape(-1)))
    np.testing.assert_array_equal(oracle.r_energy(L, 2.0 * J, s.reshape(-1)), 2.0 * E)
    assert oracle.r_energy(L, J, np.ones(N, np.int8))[0] == -math.fsum(J)


def test_exact_routes_agree_with_closed_forms(gold):
    J = pa_inputs.couplings_gauss(3, gold["coupling_seed"])
    assert gold["sum_J2"] == pytest.approx(float((J * J).sum()), rel=1e-14)
    r0 = gold["rows"][0]
    assert r0["beta"] == 0.0
    assert r0["lnZ"] == pytest.approx(27 * math.log(2.0), rel=1e-14)       # Omega = 2^N
    assert abs(r0["mean_E"]) < 1e-9                                         # <E>_inf = 0
    assert r0["var_E"] == pytest.approx(float((J * J).sum()), rel=1e-10)    # sum_b J_b^2
    for r in gold["rows"]:
        assert r["lnZ"] == pytest.approx(r["lnZ_transfer"], rel=1e-12, abs=1e-10)
        assert r["mean_E"] == pytest.approx(r["mean_E_transfer"], rel=1e-10, abs=1e-10)
    # d lnZ / d beta = -<E>: finite differences of the exact lnZ
    tm = TransferMatrixL3(J)
    for b in (0.3, 1.0, 2.0):
        h = 1e-5
        d = (tm.lnZ(b + h) - tm.lnZ(b - h)) / (2 * h)
        assert d == pytest.approx(-tm.mean_energy(b), rel=1e-6)
    # the ground state bounds <E> from below and is approached at large beta
    assert all(r["mean_E"] >= gold["E0"] - 1e-9 for r in gold["rows"])
    assert gold["rows"][-1]["mean_E"] - gold["E0"] < 1.0


def test_thresholds():
    assert oracle.lib().pao_r_threshold(0.7, 0.0) == 2 ** 32
    assert oracle.lib().pao_r_threshold(0.7, -3.5) == 2 ** 32
    assert oracle.lib().pao_r_threshold(0.0, 5.0) == 2 ** 32
    assert oracle.lib().pao_r_threshold(1e6, 0.5) == 0
    for beta, dE in ((0.3, 1.7), (1.1, 0.25), (2.0, 4.0)):
        t = oracle.lib().pao_r_threshold(beta, dE)
        assert t == math.floor(math.ldexp(oracle.r_exp(-beta * dE)[0], 32))
        assert abs(t - math.ldexp(math.exp(-beta * dE), 32)) <= 2.0


def _thresholds_agree_pm(beta):
    thr = oracle.thresholds(beta)
    return all(oracle.lib().pao_r_threshold(beta, 4.0 * (i + 1)) == int(thr[i]) for i in range(3))


@pytest.mark.parametrize("beta", [0.0, 0.2, 0.45, 1.3])
def test_sweep_reduces_to_pm_sweep(beta):
    """With J = +-1 every threshold equals the +-J one (checked), so the sweep
    must reproduce the +-J oracle's sweep bit for bit."""
    assert _thresholds_agree_pm(beta)
    L, R = 4, 300
    N = L ** 3
    J = pa_inputs.couplings_pm(L, 31)
    p = oracle.Population(L, J, R, 77)
    g = oracle.GaussRealPopulation(L, J.astype(np.float64), R, 77)
    np.testing.assert_array_equal(g.spins, p.spins)
    np.testing.assert_array_equal(g.U, (2 * p.U - 3 * N).astype(np.float64))
    p.sweep(beta, 7)
    g.sweep(beta, 7)
    np.testing.assert_array_equal(g.spins, p.spins)
    np.testing.assert_array_equal(g.U, (2 * p.U - 3 * N).astype(np.float64))


@pytest.mark.parametrize("beta", [0.15, 0.6])
def test_sweep_reduces_to_quantised_sweep(beta):
    """With J = k/16 (on the grid) the sweep reproduces the 1/16-quantised
    oracle wherever the two threshold tables agree (checked for every dE16)."""
    L, R = 4, 200
    K = pa_inputs.couplings_gauss16(L, 41)
    dEmax = oracle.g_dE_max(L, K)
    gthr = oracle.g_thresholds(beta, dEmax)
    assert all(oracle.lib().pao_r_threshold(beta, d / 16.0) == int(gthr[d])
               for d in range(1, dEmax + 1))
    q = oracle.GaussPopulation(L, K, R, 5)
    g = oracle.GaussRealPopulation(L, K / 16.0, R, 5)
    q.sweep(beta, 5)
    g.sweep(beta, 5)
    np.testing.assert_array_equal(g.spins, q.spins)
    np.testing.assert_array_equal(g.U, q.U / 16.0)


def test_beta_zero_sweep_flips_every_spin_and_tracks_energy():
    L, R = 4, 50
    J = pa_inputs.couplings_gauss(L, 3)
    g = oracle.GaussRealPopulation(L, J, R, 9)
    s0 = g.spins.copy()
    g.sweep(0.0, 1)
    np.testing.assert_array_equal(g.spins, -s0)
    g.sweep(0.8, 4)
    np.testing.assert_array_equal(g.U, oracle.r_energy(L, J, g.spins))


def test_zero_temperature_never_raises_energy():
    L, R = 4, 64
    J = pa_inputs.couplings_gauss(L, 8)
    g = oracle.GaussRealPopulation(L, J, R, 2)
    prev = g.U.copy()
    for _ in range(5):
        g.sweep(1e6, 1)
        assert np.all(g.U <= prev)
        prev = g.U.copy()
    np.testing.assert_array_equal(g.U, oracle.r_energy(L, J, g.spins))


def test_metropolis_samples_boltzmann_l3(gold):
    J = pa_inputs.couplings_gauss(3, gold["coupling_seed"])
    row = [r for r in gold["rows"] if r["beta"] == 0.6][0]
    R = 20000
    g = oracle.GaussRealPopulation(3, J, R, 21)
    g.sweep(0.6, 200)
    np.testing.assert_array_equal(g.U, oracle.r_energy(3, J, g.spins))
    m, v = float(g.U.mean()), float(g.U.var())
    assert abs(m - row["mean_E"]) < 5 * math.sqrt(row["var_E"] / R), (m, row)
    assert abs(v - row["var_E"]) < 0.1 * row["var_E"], (v, row)


def test_fixed_point_sum_is_the_exact_sum_of_truncated_terms():
    rng = np.random.default_rng(3)
    for v in (rng.uniform(0, 1, 5000), np.exp(-rng.uniform(0, 80, 5000)),
              np.concatenate([np.ones(3), np.ldexp(rng.uniform(0.5, 1, 100), -rng.integers(
                  40, 120, 100)), np.zeros(5)])):
        want = sum(int(math.ldexp(float(x), 96)) for x in v)   # floor: x >= 0
        assert oracle.r_fixsum96(v) == want
        S = oracle.r_round96(want)
        assert S == float(want) / 2.0 ** 96
        # within R 2^-96 of the exact sum, so equal to the correctly rounded one here
        assert S == math.fsum(v.tolist())
    assert oracle.r_fixsum96(np.ones(1000)) == 1000 << 96


def test_resampling_reduces_to_the_pm_table():
    """J = +-1 as reals: weights, S and the copy counts of the +-J table (level
    form, its own exp and sequential sum) agree: the counts exactly, S and ln Q
    to a few ulps."""
    L, R = 4, 3000
    N = L ** 3
    J = pa_inputs.couplings_pm(L, 15)
    p = oracle.Population(L, J, R, 5)
    g = oracle.GaussRealPopulation(L, J.astype(np.float64), R, 5)
    p.sweep(0.6, 5)
    g.sweep(0.6, 5)
    for b in (0.65, 0.8, 1.2):
        p.resample(b)
        g.resample(b)
        np.testing.assert_array_equal(g.last["n"], p.last["n"])
        assert g.last["lnQ"] == pytest.approx(p.last["lnQ"], rel=1e-13, abs=1e-14)
        assert g.last["eps"] == pytest.approx(p.last["eps"], rel=1e-12, abs=1e-15)
        np.testing.assert_array_equal(g.fam, p.fam)
        np.testing.assert_array_equal(g.U, (2 * p.U - 3 * N).astype(np.float64))
        p.sweep(b, 2)
        g.sweep(b, 2)


def test_identity_resampling_at_zero_step():
    L, R = 4, 500
    g = oracle.GaussRealPopulation(L, pa_inputs.couplings_gauss(L, 1), R, 3)
    g.sweep(0.5, 3)
    s, f = g.spins.copy(), g.fam.copy()
    g.resample(g.beta)             # dbeta = 0 (beta is still 0 here)
    assert g.last["S"] == float(R)
    assert np.all(g.last["n"] == 1) and g.last["lnQ"] == 0.0 and g.last["eps"] == 0.0
    np.testing.assert_array_equal(g.spins, s)
    np.testing.assert_array_equal(g.fam, f)


def test_copy_counts_mean_and_conservation():
    L, R = 4, 20000
    g = oracle.GaussRealPopulation(L, pa_inputs.couplings_gauss(L, 2), R, 4)
    g.sweep(0.3, 3)
    g.resample(0.5)
    n, tau = g.last["n"].astype(np.float64), g.last["tau"]
    assert math.fsum(tau) == pytest.approx(R, rel=1e-12)          # sum tau = R (Eq. 1)
    assert np.all((n == np.floor(tau)) | (n == np.floor(tau) + 1))
    assert abs(n.sum() - R) < 5 * math.sqrt(R)
    # E[n - floor tau] = frac tau, each replica a Bernoulli draw
    fr = tau - np.floor(tau)
    assert abs((n - np.floor(tau)).sum() - fr.sum()) < 5 * math.sqrt((fr * (1 - fr)).sum())


def test_constant_culling_bisection():
    L, R = 4, 5000
    g = oracle.GaussRealPopulation(L, pa_inputs.couplings_gauss(L, 6), R, 8)
    g.sweep(0.0, 2)
    eps = 0.1
    b = g.choose_beta(eps, 5.0)
    d = b - g.beta
    E = g.U[: g.R_tilde]
    assert oracle.r_culling_fraction(E, R, d) <= eps
    assert oracle.r_culling_fraction(E, R, math.nextafter(d, 10.0) * (1 + 1e-12)) > eps
    # the Gaussian estimate of Sec. III.C: eps ~ dbeta sigma_E / sqrt(2 pi)
    est = eps * math.sqrt(2 * math.pi) / float(E.std())
    assert 0.7 * est < d < 1.3 * est, (d, est)
    # the whole remaining range is taken when it culls no more than the target
    assert g.choose_beta(0.9999, g.beta + 1e-9) == g.beta + 1e-9


def test_pa_matches_exact_l3(gold):
    """Linear schedule to beta = 2 at L = 3: beta F (Eq. 9) and <E> within their
    statistical errors of the exact values at every golden temperature."""
    J = pa_inputs.couplings_gauss(3, gold["coupling_seed"])
    R = 20000
    g = oracle.GaussRealPopulation(3, J, R, 101)
    betas = oracle.linear_schedule(2.0, 41)
    want = {round(r["beta"], 10): r for r in gold["rows"]}
    checked = 0
    for k in range(1, len(betas)):
        g.resample(betas[k])
        g.sweep(betas[k], 10)
        r = g.observables()
        w = want.get(round(betas[k], 10))
        if w is None:
            continue
        checked += 1
        np.testing.assert_array_equal(g.U, oracle.r_energy(3, J, g.spins))
        sig = math.sqrt(max(r.rho_t - 1.0, 1e-3) / R)
        assert abs(r.beta_F - (-w["lnZ"])) <= 5 * sig + max(r.rho_t - 1, 0) / (2 * R), (k, r)
        assert abs(r.mean_E - w["mean_E"]) <= 5 * math.sqrt(w["var_E"] * r.rho_t / R) + 1e-9
    assert checked == 11


def test_adaptive_pa_matches_transfer_matrix_l3(gold):
    """Constant-culling schedule (Sec. III.C) at L = 3 to beta = 1.5: every step
    within statistical error of the transfer-matrix lnZ and <E> at its beta."""
    J = pa_inputs.couplings_gauss(3, gold["coupling_seed"])
    tm = TransferMatrixL3(J)
    R = 10000
    g = oracle.GaussRealPopulation(3, J, R, 202)
    steps = 0
    while g.beta < 1.5 and steps < 200:
        b = g.choose_beta(0.1, 1.5)
        g.resample(b)
        g.sweep(b, 10)
        r = g.observables()
        steps += 1
        assert r.eps_expected <= 0.1 + 1e-15
        sig = math.sqrt(max(r.rho_t - 1.0, 1e-3) / R)
        assert abs(r.beta_F + tm.lnZ(b)) <= 5 * sig + max(r.rho_t - 1, 0) / (2 * R), (steps, r)
    assert g.beta == 1.5 and 5 < steps < 200
