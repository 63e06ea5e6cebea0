"""Pins for the CPU oracle: checks against facts that do not come from the
oracle itself (a library generator, exact enumeration, a second exact method,
closed forms and special cases, the paper's statistical laws).

Paper: Amey & Machta, arXiv:1711.02146.  Each test names the passage it
checks.  Statistical tests use fixed seeds and bands set from the paper's own
error statements (Sec. III.A error bound on an observable, the rho_f <= rho_t - 1
inequality of Sec. III.B, the free-energy bias of Sec. V.E).
"""
import json
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import pa_inputs
from oracle.exact import TransferMatrixL3, thermo_from_dos

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "l3_exact.json")


@pytest.fixture(scope="module")
def l3():
    with open(GOLD) as f:
        d = json.load(f)
    J = pa_inputs.couplings_pm(3, d["coupling_seed"])
    return d, J


# ---------------------------------------------------------------------------
# Philox4x32-10 against rocRAND's engine (Salmon et al. SC'11 generator)
# ---------------------------------------------------------------------------
def test_philox_matches_rocrand_engine(oracle_lib, tmp_path):
    gxx = shutil.which("g++")
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    assert gxx and os.path.exists(hdr), "g++ and rocRAND headers are needed for this pin"
    exe = tmp_path / "philox_ref"
    subprocess.check_call([gxx, "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", str(exe)])
    rng = np.random.default_rng(11)
    cases = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6,
             [0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344, 0xA4093822, 0x299F31D0]]
    cases += rng.integers(0, 2 ** 32, size=(300, 6), dtype=np.uint64).tolist()
    # the counters the method actually uses: (slot, sweep, cm>>2, tag) etc.
    for r in (0, 1, 499999):
        for tag in (0x494E4954, 0x4D455452, 0x52455341):
            cases.append([r, 7, 3, tag, 0x5EED0001, 0])
    text = "".join(" ".join("%x" % v for v in c) + "\n" for c in cases)
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout
    ref = [[int(w, 16) for w in line.split()] for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, want in zip(cases, ref):
        got = oracle.philox(c[:4], c[4:])
        assert [int(x) for x in got] == want, c


# ---------------------------------------------------------------------------
# Lattice (Sec. II.A): periodic cubic lattice, each bond once
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [3, 4, 6, 10])
def test_lattice_tables(oracle_lib, L):
    N = L ** 3
    nb, bd = oracle.neighbours(L)
    opposite = [1, 0, 3, 2, 5, 4]
    for s in range(N):
        for d in range(6):
            assert nb[nb[s, d], opposite[d]] == s
            assert bd[s, d] == bd[nb[s, d], opposite[d]]  # same bond seen from both ends
    counts = np.bincount(bd.ravel(), minlength=3 * N)
    assert np.all(counts == 2)  # 3N bonds, each touching two sites
    cm = oracle.colour_major(L)
    assert sorted(cm.tolist()) == list(range(N))
    if L % 2 == 0:
        x, y, z = np.arange(N) % L, (np.arange(N) // L) % L, np.arange(N) // (L * L)
        c = (x + y + z) & 1
        # even L: the rank among same-colour sites is site >> 1
        assert np.array_equal(cm, c * (N // 2) + (np.arange(N) >> 1))
        # checkerboard: no bond joins two sites of the same colour
        assert np.all(c[nb] != c[:, None])


# ---------------------------------------------------------------------------
# Energy special cases and the exact density of states
# ---------------------------------------------------------------------------
def test_energy_special_cases(oracle_lib):
    for L in (3, 4, 6):
        N = L ** 3
        up = np.ones(N, np.int8)
        ferro = pa_inputs.couplings_ferro(L)
        assert oracle.energy(L, ferro, up)[0] == 0  # E = -3N ground state
        J = pa_inputs.couplings_pm(L, 99 + L)
        # all spins up: exactly the antiferromagnetic bonds are unsatisfied
        assert oracle.energy(L, J, up)[0] == np.count_nonzero(J < 0)
        rng = np.random.default_rng(L)
        s = (1 - 2 * rng.integers(0, 2, size=(50, N))).astype(np.int8)
        U = oracle.energy(L, J, s.ravel())
        assert np.array_equal(U, oracle.energy(L, J, (-s).ravel()))  # global flip symmetry
        assert np.all((U >= 0) & (U <= 3 * N))


def test_density_of_states_closed_forms(oracle_lib, l3):
    d, J = l3
    N = 27
    g = np.array(d["dos"], dtype=np.float64)
    assert np.array_equal(np.array(d["dos"], np.uint64), oracle.density_of_states(3, J))
    assert g.sum() == 2.0 ** N
    U = np.arange(g.size)
    # beta = 0: every bond is unsatisfied in exactly half of the states, and
    # the bond indicators are pairwise independent: mean 3N/2, variance 3N/4
    assert (g * U).sum() / 2.0 ** N == pytest.approx(1.5 * N, rel=1e-15)
    var = (g * U * U).sum() / 2.0 ** N - (1.5 * N) ** 2
    assert var == pytest.approx(0.75 * N, rel=1e-12)
    # ferromagnet: 2 ground states, 2N states with one flipped spin (U = 6)
    gf = oracle.density_of_states(3, pa_inputs.couplings_ferro(3))
    assert gf[0] == 2 and gf[6] == 2 * N and gf[1:6].sum() == 0


def test_two_exact_routes_agree(oracle_lib, l3):
    d, J = l3
    g = np.array(d["dos"], dtype=np.uint64)
    tm = TransferMatrixL3(J)
    for row in d["rows"]:
        b = row["beta"]
        lnZ, Em, vE = thermo_from_dos(g, 27, b)
        assert lnZ == pytest.approx(row["lnZ"], rel=1e-13)
        assert tm.lnZ(b) == pytest.approx(lnZ, rel=1e-12)
        C = tm.correlations(b)
        assert tm.mean_energy(b, C) == pytest.approx(Em, abs=1e-9)
        assert np.allclose(np.diag(C), 1.0)
    assert tm.q2(0.0) == pytest.approx(1.0 / 27.0, rel=1e-12)  # independent spins
    tf = TransferMatrixL3(pa_inputs.couplings_ferro(3))
    assert tf.q2(8.0) == pytest.approx(1.0, abs=1e-9)  # ordered ferromagnet


# ---------------------------------------------------------------------------
# Metropolis (the MCMC step of Sec. II)
# ---------------------------------------------------------------------------
def test_thresholds_limits(oracle_lib):
    assert [int(x) for x in oracle.thresholds(0.0)] == [2 ** 32] * 3
    assert [int(x) for x in oracle.thresholds(100.0)] == [0, 0, 0]
    prev = oracle.thresholds(0.0)
    for b in np.linspace(0.01, 3, 50):
        t = oracle.thresholds(b)
        assert t[0] >= t[1] >= t[2]
        assert np.all(t <= prev)
        assert abs(int(t[0]) / 2 ** 32 - math.exp(-4 * b)) < 2.0 ** -32
        prev = t


@pytest.mark.parametrize("L", [3, 4])
def test_beta_zero_sweep_flips_every_spin(oracle_lib, L):
    J = pa_inputs.couplings_pm(L, 5)
    p = oracle.Population(L, J, 64, seed=77)
    before = p.spins.copy()
    U0 = p.U.copy()
    p.sweep(0.0, 1)
    assert np.array_equal(p.spins, -before)
    assert np.array_equal(p.U, U0)


def test_zero_temperature_never_raises_energy(oracle_lib):
    L = 4
    J = pa_inputs.couplings_pm(L, 6)
    p = oracle.Population(L, J, 200, seed=3)
    prev = p.U.copy()
    for _ in range(5):
        p.sweep(100.0, 1)
        assert np.all(p.U <= prev)
        prev = p.U.copy()
    assert np.array_equal(p.U, oracle.energy(L, J, p.spins))


def test_metropolis_samples_boltzmann_l3(oracle_lib, l3):
    """A long chain at fixed beta must reproduce the exact P(U) = g e^{-beta E}/Z."""
    d, J = l3
    g = np.array(d["dos"], dtype=np.float64)
    N = 27
    beta = 0.5
    p = oracle.Population(3, J, 20000, seed=21)
    p.sweep(beta, 200)
    assert np.array_equal(p.U, oracle.energy(3, J, p.spins))  # incremental == recomputed
    h = np.bincount(p.U, minlength=g.size).astype(np.float64)
    E = 2.0 * np.arange(g.size) - 3 * N
    logw = np.where(g > 0, np.log(np.maximum(g, 1)) - beta * E, -np.inf)
    P = np.exp(logw - logw.max())
    P /= P.sum()
    expect = P * p.R
    m = expect > 5
    chi2 = (((h[m] - expect[m]) ** 2) / expect[m]).sum()
    dof = int(m.sum()) - 1
    # 20000 replicas, 200 sweeps each (far beyond equilibration at beta = 0.5)
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)
    assert h[~m].sum() < 40


# ---------------------------------------------------------------------------
# Resampling (Sec. II, Eqs. 1-2)
# ---------------------------------------------------------------------------
def _random_hist(L, R, beta, seed):
    J = pa_inputs.couplings_pm(L, seed)
    p = oracle.Population(L, J, R, seed=seed)
    p.sweep(beta, 5)
    return p


def test_table_sums_to_target_and_matches_definition(oracle_lib):
    p = _random_hist(6, 5000, 0.4, 12)
    h = p.histogram()
    N = p.N
    for dbeta in (0.0, 0.01, 0.05, 0.3):
        fl, T, tau, lnQ, jmin = oracle.table(h, N, p.R, p.R_tilde, dbeta)
        assert np.flatnonzero(h)[0] == jmin
        # sum_i tau_i = R (Eqs. 1-2)
        assert float((h * tau).sum()) == pytest.approx(p.R, rel=1e-12)
        # ln Q straight from Eq. 2 over replicas, no shift, no level grouping
        E = 2.0 * p.U.astype(np.float64) - 3 * N
        a = -dbeta * E
        direct = a.max() + math.log(np.exp(a - a.max()).sum()) - math.log(p.R_tilde)
        assert lnQ == pytest.approx(direct, abs=1e-11)
        occ = h > 0
        assert np.all(fl[occ] == np.floor(tau[occ]))
        frac = tau[occ] - np.floor(tau[occ])
        assert np.all(np.abs(T[occ].astype(np.float64) / 2.0 ** 53 - frac) <= 2.0 ** -53)


def test_identity_resampling_at_zero_step(oracle_lib):
    p = _random_hist(4, 1000, 0.3, 3)
    spins, U, fam = p.spins.copy(), p.U.copy(), p.fam.copy()
    p.resample(p.beta)  # dbeta = 0 with R~ = R: tau = 1 for everybody
    assert p.last["lnQ"] == 0.0
    assert np.all(p.last["n"] == 1)
    assert np.array_equal(p.spins, spins) and np.array_equal(p.U, U) and np.array_equal(p.fam, fam)


def test_copy_counts_mean_and_variance(oracle_lib):
    """E[n_i] = tau_i and var(R~') = sum frac (1 - frac) (Sec. II; App. B var z)."""
    p = _random_hist(6, 4000, 0.3, 8)
    h = p.histogram()
    fl, T, tau, lnQ, jmin = oracle.table(h, p.N, p.R, p.R_tilde, 0.05)
    tau_i = tau[p.U]
    trials = 400
    totals = []
    acc = np.zeros(p.R_tilde)
    for step in range(1, trials + 1):
        n = oracle.copy_counts(p.U, fl, T, p.seed, step)
        assert np.all((n == fl[p.U]) | (n == fl[p.U] + 1))
        acc += n
        totals.append(int(n.sum()))
    frac = tau_i - np.floor(tau_i)
    var_theory = float((frac * (1 - frac)).sum())
    mean_n = acc / trials
    # per-replica means: z-scores against binomial standard errors
    se = np.sqrt(np.maximum(frac * (1 - frac), 1e-12) / trials)
    z = (mean_n - tau_i) / se
    assert np.abs(z[frac > 0.01]).max() < 5.5
    assert np.mean(totals) == pytest.approx(p.R, abs=5 * math.sqrt(var_theory / trials))
    # sample variance of the total against the closed form (chi-square band)
    v = np.var(totals, ddof=1)
    assert 0.75 * var_theory < v < 1.3 * var_theory


# ---------------------------------------------------------------------------
# Whole PA runs at L = 3 against exact results (Sec. II, Eq. 9, Sec. III.A)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def pa_l3(l3):
    d, J = l3
    steps = []

    def check(k, pops):
        for p in pops:
            assert np.array_equal(p.U, oracle.energy(3, J, p.spins))  # incremental U
            assert np.all(np.diff(p.fam.astype(np.int64)) >= 0)  # labels stay sorted
            assert p.fam.max() < p.R

    pops, recs = oracle.run_linear(3, J, 20000, seed=101, beta_max=2.0, n_temps=41, n_sweeps=10,
                                   partner_seed=102, on_step=check)
    return d, J, pops, recs


def test_free_energy_at_beta_zero_is_log_omega(oracle_lib, l3):
    d, J = l3
    p = oracle.Population(3, J, 100, seed=1)
    assert p.observables().beta_F == -(27 * math.log(2.0))  # ln Omega, Omega = 2^N (Eq. 9)


def _exact_at(d, beta):
    g = np.array(d["dos"], np.uint64)
    return thermo_from_dos(g, 27, beta)


def test_pa_free_energy_and_energy_match_exact_l3(oracle_lib, pa_l3):
    d, J, pops, recs = pa_l3
    for recs_k, q in recs:
        for r in recs_k:
            lnZ, Em, vE = _exact_at(d, r.beta)
            R = 20000
            # Sec. III.B: var(beta F~) R -> rho_f <= rho_t - 1; Sec. V.E bias rho_f / (2R)
            sig = math.sqrt(max(r.rho_t - 1.0, 1e-3) / R)
            assert abs(r.beta_F - (-lnZ)) <= 5 * sig + max(r.rho_t - 1, 0) / (2 * R), r
            # Sec. III.A: delta O <= sqrt(var(O) rho_t / R)
            assert abs(r.mean_E - Em) <= 5 * math.sqrt(vE * r.rho_t / R) + 1e-9, r


def test_pa_overlap_q2_matches_exact_l3(oracle_lib, pa_l3):
    d, J, pops, recs = pa_l3
    rows = {round(x["beta"], 6): x for x in d["rows"]}
    N = 27
    checked = 0
    for recs_k, q in recs:
        b = round(recs_k[0].beta, 6)
        if b not in rows:
            continue
        # bins are distinct for N = 27, so q is recovered exactly from the bin
        dvals = np.arange(N + 1)
        bins = (128 * (N - dvals) + N) // (2 * N)
        assert len(set(bins.tolist())) == N + 1
        qv = 1.0 - 2.0 * dvals / N
        counts = np.array([q[bn] for bn in bins], np.float64)
        est = float((counts * qv ** 2).sum() / counts.sum())
        rho = max(recs_k[0].rho_t, recs_k[1].rho_t)
        assert abs(est - rows[b]["q2"]) <= 5 * math.sqrt(rho / counts.sum()) + 1e-9, (b, est)
        checked += 1
    assert checked >= 4


def test_ferromagnet_anneals_to_ground_state(oracle_lib):
    L = 4
    N = L ** 3
    pops, recs = oracle.run_linear(L, pa_inputs.couplings_ferro(L), 1000, seed=9, beta_max=5.0,
                                   n_temps=51, n_sweeps=10)
    last = recs[-1][0][0]
    assert last.E_min == -3 * N
    assert last.mean_E == -3.0 * N


# ---------------------------------------------------------------------------
# Families and the constant-culling schedule (Sec. III.A, III.C-III.E)
# ---------------------------------------------------------------------------
def _bisect_crossing(h, R, eps, rem):
    """The crossing by plain bisection (64 halvings, lower end kept), written
    here in Python over the oracle's culling fraction: the oracle's step must
    take exactly the same path."""
    lo, hi = 0.0, rem
    for _ in range(64):
        mid = lo + 0.5 * (hi - lo)
        if oracle.culling_fraction(h, R, mid) <= eps:
            lo = mid
        else:
            hi = mid
    return lo


def test_adaptive_step_bisection_and_gaussian_estimate(oracle_lib):
    p = _random_hist(6, 20000, 0.0, 4)
    h = p.histogram()
    for eps in (0.02, 0.05, 0.1):
        dbeta, end = oracle.choose_dbeta(h, p.R, eps, 5.0)
        assert not end
        assert oracle.culling_fraction(h, p.R, dbeta) <= eps
        assert oracle.culling_fraction(h, p.R, dbeta * (1 + 1e-9) + 1e-15) > eps
        assert dbeta == _bisect_crossing(h, p.R, eps, 5.0)
        # Sec. III.C: dbeta ~ eps sqrt(2 pi) / sigma_E for small dbeta sigma_E
        E = 2.0 * np.arange(h.size) - 3 * p.N
        w = h.astype(np.float64)
        m = (w * E).sum() / w.sum()
        sigma = math.sqrt((w * (E - m) ** 2).sum() / w.sum())
        approx = eps * math.sqrt(2 * math.pi) / sigma
        assert dbeta == pytest.approx(approx, rel=0.1 + 2 * eps)
    # a range that culls less than the target is taken whole
    dbeta, end = oracle.choose_dbeta(h, p.R, 0.1, 1e-6)
    assert end and dbeta == 1e-6
    # a late-anneal histogram with three occupied levels: eps(dbeta) flattens
    # out and the crossing lies far from the small-step estimate
    h3 = np.zeros(h.size, np.uint32)
    h3[[10, 11, 13]] = [15000, 4000, 1000]
    for eps in (0.05, 0.1, 0.2):
        dbeta, end = oracle.choose_dbeta(h3, 20000, eps, 5.0)
        if end:
            assert oracle.culling_fraction(h3, 20000, 5.0) <= eps
            continue
        assert oracle.culling_fraction(h3, 20000, dbeta) <= eps
        assert oracle.culling_fraction(h3, 20000, dbeta * (1 + 2.0 ** -38)) > eps
        assert dbeta == _bisect_crossing(h3, 20000, eps, 5.0)


def _plaquette_sum(L, J):
    """Sum over the 3N elementary plaquettes of the product of their four
    couplings, from the bond convention b = d N + site (site to site + e_d)."""
    N = L ** 3

    def site(x, y, z):
        return (x % L) + L * ((y % L) + L * (z % L))

    e = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
    tot = 0
    for z in range(L):
        for y in range(L):
            for x in range(L):
                s = site(x, y, z)
                for d1 in range(3):
                    for d2 in range(d1 + 1, 3):
                        a, b = e[d1], e[d2]
                        s1 = site(x + a[0], y + a[1], z + a[2])
                        s2 = site(x + b[0], y + b[1], z + b[2])
                        tot += (int(J[d1 * N + s]) * int(J[d2 * N + s1]) * int(J[d1 * N + s2])
                                * int(J[d2 * N + s]))
    return tot


def test_high_temperature_series_and_culled_count(oracle_lib):
    """A lattice too large to enumerate, L = 6, at high temperature.  With
    t = tanh(beta), Z = 2^N cosh(beta)^3N (1 + t^4 sum_p prod_p J + O(t^6)):
    closed loops of the expansion are plaquettes first (the shortest winding
    loops have length L = 6).  PA on a linear schedule to beta = 0.2 must give
    beta F~ = -ln Z and <E> = -d ln Z / d beta within its statistical error
    (Sec. II.A, Eq. 9), and at every step the realised number of culled
    replicas must match eps R, the expected count of Sec. III.C (a sum of
    independent Bernoulli(1 - tau) trials, so within 5 sqrt(eps R))."""
    L, R, bmax, n_t = 6, 30000, 0.2, 21
    N = L ** 3
    J = pa_inputs.couplings_pm(L, 5)
    P = _plaquette_sum(L, J)
    t = math.tanh(bmax)
    lnZ = N * math.log(2.0) + 3 * N * math.log(math.cosh(bmax)) + t ** 4 * P
    E_ht = -3 * N * t - 4 * t ** 3 * (1 - t * t) * P
    p = oracle.Population(L, J, R, seed=105)
    for k in range(1, n_t):
        b = bmax * k / (n_t - 1)
        p.resample(b)
        eps, culled = p.last["eps"], p.last["n_culled"]
        assert abs(culled - eps * R) <= 5 * math.sqrt(eps * R) + 1, (k, culled, eps * R)
        p.sweep(b, 10)
    r = p.observables()
    # statistics (rho_f <= rho_t - 1, Sec. III.B) plus the neglected t^6 loops
    tol_F = 4 * math.sqrt(max(r.rho_t - 1.0, 1.0) / R) + r.rho_t / (2 * R) + 0.02
    assert abs(r.beta_F + lnZ) <= tol_F, (r.beta_F, -lnZ)
    tol_E = 5 * math.sqrt(3 * N * r.rho_t / R) + 0.05
    assert abs(r.mean_E - E_ht) <= tol_E, (r.mean_E, E_ht)


def test_high_temperature_family_growth(oracle_lib):
    """MCMC-equilibrated regime, constant eps: rho_t - 1 = 2 eps k (Sec. III.E)
    and a geometric family-size law P_eta(k) (same section)."""
    L = 6
    J = pa_inputs.couplings_pm(L, 31)
    eps = 0.02
    p = oracle.Population(L, J, 20000, seed=55)
    k = 0
    while k < 25:
        b = p.choose_beta(eps, 5.0)
        p.resample(b)
        p.sweep(b, 10)
        k += 1
        assert abs(p.last["eps"] - eps) < 1e-6
    r = p.observables()
    assert r.beta < 0.2  # still deep in the high-temperature phase
    assert r.rho_t - 1.0 == pytest.approx(2 * eps * k, rel=0.1)
    sizes = oracle.family_sizes(p.fam, p.R, 12).astype(np.float64) / p.R
    ek = eps * k
    # The master equation of Sec. III.E with P_eta(0) = delta_{eta,1} is solved
    # by P_0 = ek/(1+ek), P_eta = ek^(eta-1)/(1+ek)^(eta+1): mean 1, variance
    # 2 ek.  (The printed prefactor 1/(1+ek) lacks one power and would not
    # normalise together with P_0; the variance the paper derives needs the
    # square.)
    total = ek / (1 + ek) + sum(ek ** (e - 1) / (1 + ek) ** (e + 1) for e in range(1, 400))
    assert total == pytest.approx(1.0, abs=1e-12)
    for eta in range(1, 6):
        expect = ek ** (eta - 1) / (1 + ek) ** (eta + 1)
        assert sizes[eta] == pytest.approx(expect, rel=0.1, abs=0.004)
    assert sizes[0] == pytest.approx(ek / (1 + ek), rel=0.1)


# ---------------------------------------------------------------------------
# Link overlap q_l (Sec. II.A): configurations whose bond count D is known by
# construction, and the identity D(a, b) = unsatisfied bonds of a*b in the
# ferromagnet, which goes through the oracle's separately written energy
# (itself pinned by exact enumeration above)
# ---------------------------------------------------------------------------
def _flip(s, L, *sites):
    t = s.copy()
    for (x, y, z) in sites:
        t[x + L * (y + L * z)] *= -1
    return t


@pytest.mark.parametrize("L", [3, 4, 6])
def test_link_overlap_known_configurations(oracle_lib, L):
    N = L ** 3
    rng = np.random.default_rng(L)
    a = rng.choice(np.array([-1, 1], np.int8), N)
    x, y, z = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    stagger = np.where((x + y + z) % 2 == 0, 1, -1).astype(np.int8)
    stagger = stagger.transpose(2, 1, 0).reshape(-1)  # index x + L (y + L z)
    cases = [
        (a, 0),                                              # the same configuration: q_l = 1
        (-a, 0),                                             # global flip: q_l = 1
        (_flip(a, L, (1, 1, 1)), 6),                         # one spin: its six bonds
        (_flip(a, L, (1, 1, 1), (2, 1, 1)), 10),             # x neighbours share one bond
        (_flip(a, L, (1, 1, 1), (1, 2, 1)), 10),             # y neighbours
        (_flip(a, L, (1, 1, 1), (1, 1, 2)), 10),             # z neighbours
        (_flip(a, L, (0, 1, 1), (L - 1, 1, 1)), 10),         # x neighbours across the boundary
        (_flip(a, L, (1, 0, 1), (1, L - 1, 1)), 10),         # y across the boundary
        (_flip(a, L, (1, 1, 0), (1, 1, L - 1)), 10),         # z across the boundary
    ]
    if L >= 4:
        cases.append((_flip(a, L, (0, 0, 0), (2, 2, 2)), 12))  # two far apart: 6 + 6
    if L % 2 == 0:
        cases.append((a * stagger, 3 * N))                   # staggered: every bond, q_l = -1
    A = np.stack([a] * len(cases))
    B = np.stack([c for c, _ in cases])
    hist, D = oracle.link_overlap(L, A.reshape(-1), B.reshape(-1))
    assert D.tolist() == [d for _, d in cases]
    assert int(hist.sum()) == len(cases) and hist.size == 3 * N + 1
    q_l = 1.0 - 2.0 * D / (3 * N)
    assert q_l[0] == 1.0 and q_l[1] == 1.0
    if L % 2 == 0:
        assert q_l[-1] == -1.0


@pytest.mark.parametrize("L", [4, 5, 8])
def test_link_overlap_is_ferro_energy_of_product(oracle_lib, L):
    N = L ** 3
    rng = np.random.default_rng(100 + L)
    R = 64
    a = rng.choice(np.array([-1, 1], np.int8), (R, N))
    b = rng.choice(np.array([-1, 1], np.int8), (R, N))
    _, D = oracle.link_overlap(L, a.reshape(-1), b.reshape(-1))
    ferro = np.ones(3 * N, np.int8)
    U = oracle.energy(L, ferro, (a * b).reshape(-1))
    np.testing.assert_array_equal(D, U)
    # a gauge transformation of both replicas leaves every bond term unchanged
    tau = rng.choice(np.array([-1, 1], np.int8), N)
    _, Dg = oracle.link_overlap(L, (a * tau).reshape(-1), (b * tau).reshape(-1))
    np.testing.assert_array_equal(Dg, D)
    # unequal population sizes: the first min(Ra, Rb) pairs
    hist, Dm = oracle.link_overlap(L, a[:40].reshape(-1), b.reshape(-1))
    np.testing.assert_array_equal(Dm, D[:40])
    assert int(hist.sum()) == 40
