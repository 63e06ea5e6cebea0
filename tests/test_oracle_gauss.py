"""Pins of the oracle's Gaussian-coupling path (CPU).

Couplings J = k / 16 with k = round(16 z), z a unit normal (Sec. II.A draws J
from a unit normal; the rounding keeps the energy levels integer).  The
oracle is checked against: closed forms of the exact density of states, a
second exact route (the L = 3 transfer matrix), special configurations, the
Boltzmann law of its Metropolis chain, and whole PA runs at L = 3 against the
exact free energy and energy (Amey & Machta, arXiv:1711.02146, Sec. II,
Eq. 9, Sec. III.A)."""
import math

import numpy as np
import pytest

import oracle
import pa_inputs
from oracle.exact import TransferMatrixL3, thermo_from_levels

L3_SEED = 4321


@pytest.fixture(scope="module")
def g3():
    K = pa_inputs.couplings_gauss16(3, L3_SEED)
    g, off = oracle.g_density_of_states(3, K)
    E = (np.arange(g.size, dtype=np.float64) - off) / 16.0
    return K, g, off, E


def test_couplings_are_rounded_unit_normals():
    K = pa_inputs.couplings_gauss16(10, 3).astype(np.float64)
    J = K / 16.0
    assert K.min() >= -127 and K.max() <= 127
    assert abs(J.mean()) < 0.05 and abs(J.var() - 1.0 - 1.0 / (12 * 256)) < 0.06


def test_energy_special_cases():
    L = 4
    N = L ** 3
    K = pa_inputs.couplings_gauss16(L, 11)
    up = np.ones(N, np.int8)
    assert oracle.g_energy(L, K, up)[0] == -int(K.astype(np.int64).sum())
    rng = np.random.default_rng(5)
    s = rng.choice(np.array([-1, 1], np.int8), size=N)
    assert oracle.g_energy(L, K, s)[0] == oracle.g_energy(L, K, -s)[0]   # global flip
    ferro = np.full(3 * N, 16, np.int8)
    assert oracle.g_energy(L, ferro, up)[0] == -3 * N * 16                 # E = -3N
    # with k = +-16 the energy is 16 times the +-J energy of the same signs
    Jpm = pa_inputs.couplings_pm(L, 12)
    U = oracle.energy(L, Jpm, s)[0]
    assert oracle.g_energy(L, (16 * Jpm).astype(np.int8), s)[0] == 16 * (2 * U - 3 * N)


def test_density_of_states_closed_forms(g3):
    K, g, off, E = g3
    gf = g.astype(np.float64)
    assert int(g.sum()) == 2 ** 27
    # over all states every bond term -k s s is +-k with equal weight, independently
    assert abs((gf * E).sum()) < 1e-6 * 2 ** 27
    var16 = (gf * (E * 16.0) ** 2).sum() / 2 ** 27
    assert var16 == pytest.approx(float((K.astype(np.float64) ** 2).sum()), rel=1e-12)


def test_two_exact_routes_agree(g3):
    K, g, off, E = g3
    tm = TransferMatrixL3(K.astype(np.float64) / 16.0)
    for beta in (0.0, 0.3, 1.0, 2.5):
        lnZ, Em, _ = thermo_from_levels(g, E, beta)
        assert lnZ == pytest.approx(tm.lnZ(beta), rel=1e-10, abs=1e-10)
        assert Em == pytest.approx(tm.mean_energy(beta), rel=1e-8, abs=1e-8)


def test_thresholds():
    t0 = oracle.g_thresholds(0.0, 1524)
    assert np.all(t0 == 1 << 32)
    t = oracle.g_thresholds(0.7, 1524)
    assert t[0] == 1 << 32 and np.all(np.diff(t.astype(np.float64)) <= 0)
    for d in (2, 30, 200):
        x = math.ldexp(math.exp(-0.7 * d / 16.0), 32)
        assert abs(float(t[d]) - x) <= 1.0
    assert np.all(oracle.g_thresholds(1e6, 100)[1:] == 0)


def test_beta_zero_sweep_flips_every_spin():
    L = 4
    K = pa_inputs.couplings_gauss16(L, 13)
    p = oracle.GaussPopulation(L, K, 300, 3)
    s0, E0 = p.spins.copy(), p.U.copy()
    p.sweep(0.0, 1)
    np.testing.assert_array_equal(p.spins, -s0)
    np.testing.assert_array_equal(p.U, E0)
    np.testing.assert_array_equal(p.U, oracle.g_energy(L, K, p.spins))


def test_zero_temperature_never_raises_energy():
    L = 4
    K = pa_inputs.couplings_gauss16(L, 14)
    p = oracle.GaussPopulation(L, K, 200, 4)
    prev = p.U.copy()
    for _ in range(5):
        p.sweep(1e6, 1)
        assert np.all(p.U <= prev)
        prev = p.U.copy()
    np.testing.assert_array_equal(p.U, oracle.g_energy(L, K, p.spins))


def test_metropolis_samples_boltzmann_l3(g3):
    K, g, off, E = g3
    beta = 0.5
    p = oracle.GaussPopulation(3, K, 20000, 21)
    p.sweep(beta, 200)
    np.testing.assert_array_equal(p.U, oracle.g_energy(3, K, p.spins))
    # levels (E16 + off) merged into bins of one energy unit (16 quanta)
    b = np.arange(g.size) // 16
    logw = np.where(g > 0, np.log(np.maximum(g, 1).astype(np.float64)) - beta * E, -np.inf)
    P = np.bincount(b, weights=np.exp(logw - logw.max()))
    P /= P.sum()
    h = np.bincount((p.U.astype(np.int64) + off) // 16, minlength=P.size).astype(np.float64)
    expect = P * p.R
    m = expect > 5
    chi2 = (((h[m] - expect[m]) ** 2) / expect[m]).sum()
    dof = int(m.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)
    assert h[~m].sum() < 60


def test_table_unit_reduces_to_pm_table():
    L, R = 4, 3000
    N = L ** 3
    J = pa_inputs.couplings_pm(L, 15)
    p = oracle.Population(L, J, R, 5)
    p.sweep(0.6, 5)
    h = p.histogram()
    for dbeta in (0.0, 0.05, 0.3):
        fl, T, tau, lnQ, jmin = oracle.table(h, N, R, R, dbeta)
        n = h.size
        fl2 = np.zeros(n, np.uint32)
        T2 = np.zeros(n, np.uint64)
        tau2 = np.zeros(n, np.float64)
        lnq2 = __import__("ctypes").c_double(0.0)
        # E = 2U - 3N = 2 (U - 3N/2): unit 2, lowest level at -3N/2
        j2 = oracle.lib().pao_table_unit(h, n, 2.0, -3 * N // 2, R, R, dbeta, fl2, T2, tau2,
                                         __import__("ctypes").byref(lnq2))
        assert j2 == jmin
        np.testing.assert_array_equal(fl, fl2)
        np.testing.assert_array_equal(T, T2)
        assert lnQ == lnq2.value


def test_pa_matches_exact_l3(g3):
    K, g, off, E = g3
    R = 20000
    p = oracle.GaussPopulation(3, K, R, 101)
    betas = oracle.linear_schedule(2.0, 41)
    for k in range(1, len(betas)):
        p.resample(betas[k])
        p.sweep(betas[k], 10)
        r = p.observables()
        np.testing.assert_array_equal(p.U, oracle.g_energy(3, K, p.spins))
        lnZ, Em, vE = thermo_from_levels(g, E, betas[k])
        sig = math.sqrt(max(r.rho_t - 1.0, 1e-3) / R)
        assert abs(r.beta_F - (-lnZ)) <= 5 * sig + max(r.rho_t - 1, 0) / (2 * R), (k, r)
        assert abs(r.mean_E - Em) <= 5 * math.sqrt(vE * r.rho_t / R) + 1e-9, (k, r)
