"""GPU parity for quantised Gaussian couplings (J = k / 16, Sec. II.A draws J
from a unit normal): the HIP library against the oracle's Gaussian path.

Bit-exact on spins, E16 energies, family labels, copy counts and offsets; the
FP64 scalars come from identical integers and operation orders, so they are
equal.  Amey & Machta, arXiv:1711.02146: Sec. II loop, Eqs. 1-2, Eq. 9,
Sec. III.A, Sec. III.C.
"""
import sys

import numpy as np
import pytest

import oracle
import props
import pa_inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pam():
    import torch

    assert torch.cuda.is_available()
    import paper_1711_02146_amd as m

    m.lib()
    return m


def pair(pam, L, R, seed, layout, cseed, capacity=0):
    K = pa_inputs.couplings_gauss16(L, cseed)
    g = pam.Population(L, R, K, seed, capacity=capacity, layout=layout, model="gauss16")
    o = oracle.GaussPopulation(L, K, R, seed, capacity=capacity or None)
    return K, g, o


def assert_state(g, o, what=""):
    s, u, f = g.export_state()
    assert s.shape[0] == o.R_tilde, what
    np.testing.assert_array_equal(s.reshape(-1), o.spins, err_msg="spins " + what)
    np.testing.assert_array_equal(u.view(np.int32), o.U, err_msg="E16 " + what)
    np.testing.assert_array_equal(f, o.fam, err_msg="family " + what)


def compare_obs(go, r, k):
    for key in ("beta", "dbeta", "lnQ", "beta_F", "mean_E", "rho_t", "eps_expected"):
        assert go[key] == getattr(r, key), (k, key, go[key], getattr(r, key))
    for key in ("R_tilde", "E_min", "n_culled", "sum_eta2", "n_at_E_min"):
        assert go[key] == getattr(r, key), (k, key, go[key], getattr(r, key))
    assert go["step"] == r.k


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("L,R", [(4, 1000), (6, 77), (8, 129), (10, 333), (12, 64), (16, 65)])
def test_init_parity(pam, layout, L, R):
    say("gauss init", layout, L, R)
    K, g, o = pair(pam, L, R, 0x5EED0000 + L, layout, 31 + L)
    assert_state(g, o, f"init L={L} R={R}")
    g.close()


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("beta", [0.0, 0.3, 1.0, 5.0])
def test_sweep_parity(pam, layout, beta):
    L, R = 8, 300
    say("gauss sweep", layout, beta)
    K, g, o = pair(pam, L, R, 1234, layout, 5)
    for n in (3, 2):
        g.sweep(beta, n)
        o.sweep(beta, n)
        assert_state(g, o, f"after sweeps at beta={beta}")
    g.close()


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
def test_linear_run_l4_every_step(pam, layout):
    L, R = 4, 1000
    K, g, o = pair(pam, L, R, 77, layout, 11)
    betas = oracle.linear_schedule(5.0, 51)
    for k in range(1, 51):
        g.resample(betas[k])
        o.resample(betas[k])
        c, off = g.export_counts()
        np.testing.assert_array_equal(c, o.last["n"], err_msg=f"counts step {k}")
        np.testing.assert_array_equal(off.astype(np.uint64), o.last["offsets"])
        g.sweep(betas[k], 10)
        o.sweep(betas[k], 10)
        compare_obs(g.observables(), o.observables(), k)
        if k % 10 == 0:
            assert_state(g, o, f"step {k}")
    g.close()


def test_adaptive_prefix_l10_bitpack(pam):
    L, R = 10, 2000
    K, g, o = pair(pam, L, R, 808, "bitpack64", 12)
    for k in range(1, 16):
        bg = g.choose_beta(0.1, 5.0)
        bo = o.choose_beta(0.1, 5.0)
        assert bg == bo, (k, bg, bo)
        g.resample(bg)
        o.resample(bo)
        g.sweep(bg, 10)
        o.sweep(bo, 10)
        compare_obs(g.observables(), o.observables(), k)
    assert_state(g, o, "adaptive prefix")
    g.close()


def test_adaptive_steps_many_levels_l8(pam):
    """Twenty constant-culling steps at L = 8, R = 2e4, where about 1700 levels
    are occupied at every step: the host's step choice evaluates three
    halvings' candidates at once on worker threads there, and every chosen
    beta, every step's observables and the final population must still equal
    the oracle's sequential search."""
    L, R = 8, 20000
    K, g, o = pair(pam, L, R, 0x5EED0031, "bitpack64", 31)
    for k in range(1, 21):
        lo, _ = o.window()
        occupied = int(np.count_nonzero(np.bincount(o.U[: o.R_tilde] - lo)))
        assert occupied >= 512, (k, occupied)
        bg = g.choose_beta(0.1, 5.0)
        bo = o.choose_beta(0.1, 5.0)
        assert bg == bo, (k, bg, bo)
        g.resample(bg)
        o.resample(bo)
        g.sweep(bg, 10)
        o.sweep(bo, 10)
        compare_obs(g.observables(), o.observables(), k)
    assert_state(g, o, "adaptive steps, many levels")
    g.close()


@pytest.mark.parametrize("L,R", [(4, 140000), (6, 5000)])
def test_sweep_forms_parity(pam, L, R):
    K, g, o = pair(pam, L, R, 4321 + R, "bitpack64", 9 + L)
    for b in (0.4, 0.8):
        g.resample(b)
        o.resample(b)
        g.sweep(b, 2)
        o.sweep(b, 2)
        assert_state(g, o, f"L={L} R={R} beta={b}")
    g.close()


def test_two_populations_overlap(pam):
    L, R = 8, 2000
    K = pa_inputs.couplings_gauss16(L, 21)
    ga = pam.Population(L, R, K, 1, model="gauss16")
    gb = pam.Population(L, R, K, 2, model="gauss16")
    oa = oracle.GaussPopulation(L, K, R, 1)
    ob = oracle.GaussPopulation(L, K, R, 2)
    betas = oracle.linear_schedule(3.0, 11)
    for k in range(1, 11):
        for g, o in ((ga, oa), (gb, ob)):
            g.resample(betas[k])
            o.resample(betas[k])
            g.sweep(betas[k], 5)
            o.sweep(betas[k], 5)
        q, _ = oracle.overlap_hist(L ** 3, oa.spins, ob.spins)
        np.testing.assert_array_equal(pam.overlap_hist(ga, gb), q)
    ga.close()
    gb.close()


@pytest.mark.parametrize("split", [4, 8])
def test_full_size_l10_sampled_first_step(pam, split):
    """The benchmark's Gaussian workload, L = 10, R = 5e5, bit-packed, constant
    culling, in each sweep form its autotuner may pick: the first step in full
    (counts, offsets, labels) and 192 sampled replicas swept by the oracle."""
    L, R = 10, 500000
    N = L ** 3
    K = pa_inputs.couplings_gauss16(L, 3)
    pam.pa_autotune_reset()
    pam.pa_autotune_set(L, R, split, layout="bitpack64", model="gauss16")
    g = pam.Population(L, R, K, 42, layout="bitpack64", model="gauss16")
    o = oracle.GaussPopulation(L, K, R, 42)
    s, u, f = g.export_state()
    np.testing.assert_array_equal(s.reshape(-1), o.spins)
    np.testing.assert_array_equal(u.view(np.int32), o.U)
    del s
    bg = g.choose_beta(0.1, 5.0)
    bo = o.choose_beta(0.1, 5.0)
    assert bg == bo
    g.resample(bg)
    o.resample(bo)
    n = o.last["n"]
    c, off = g.export_counts()
    np.testing.assert_array_equal(c, n)
    np.testing.assert_array_equal(off.astype(np.uint64), o.last["offsets"])
    Rn = int(n.sum())
    g.sweep(bg, 10)
    s2, u2, f2 = g.export_state()
    assert s2.shape[0] == Rn
    np.testing.assert_array_equal(f2, o.fam)
    rng = np.random.default_rng(7)
    pick = np.unique(np.concatenate([rng.integers(0, Rn, 192), [0, Rn - 1]]))
    sp = o.spins.reshape(Rn, N)[pick].copy()
    E = o.U[pick].copy()
    oracle.g_sweep_slots(L, K, sp, E, pick.astype(np.uint32), o.seed, bo, 0, 10)
    np.testing.assert_array_equal(s2[pick], sp)
    np.testing.assert_array_equal(u2[pick].view(np.int32), E)
    np.testing.assert_array_equal(u2.view(np.int32), props.energy16(L, K, s2))
    assert g.observables()["R_tilde"] == Rn
    g.close()
    pam.pa_autotune_reset()


def test_gauss_rejected_by_batches_and_steppers(pam):
    import torch

    stream = torch.cuda.Stream()
    K = pa_inputs.couplings_gauss16(4, 1)
    g = pam.Population(4, 300, K, 1, model="gauss16", stream=stream)
    st = pam.Stepper(2, 4, stream)
    with pytest.raises(pam.PAError) as e:
        st.step([g], [0.1], [1])
    assert e.value.status == pam.PA_EINVAL
    with pytest.raises(pam.PAError) as e:
        pam.Batch([g], [0.0, 0.1], 1)
    assert e.value.status == pam.PA_EINVAL
    # out-of-range couplings are refused
    with pytest.raises(pam.PAError):
        pam.Population(4, 300, np.full(192, -128, np.int8), 1, model="gauss16")
    st.close()
    g.close()


def test_import_state_roundtrip(pam):
    """A state built by the oracle, imported (E16 recomputed on the GPU), swept on both sides."""
    L, R = 8, 200
    K = pa_inputs.couplings_gauss16(L, 12)
    o = oracle.GaussPopulation(L, K, R, 4242)
    o.sweep(0.7, 3)
    g = pam.Population(L, R, K, 4242, layout="bitpack64", model="gauss16")
    g.import_state(o.spins.reshape(R, -1), o.fam, o.t, o.k, o.beta, o.sum_lnQ)
    assert_state(g, o, "imported")
    g.sweep(0.9, 2)
    o.sweep(0.9, 2)
    assert_state(g, o, "imported + swept")
    g.close()


def test_full_anneal_l10_r500k(pam):
    """The benchmark anneal with Gaussian couplings, every step (~300) checked
    against properties that hold at any size, and the final population too:
    the E16 of sampled replicas against the energy of their exported spins
    (tests/props.py), the step record against the exported population."""
    import math

    L, R, eps, bmax = 10, 500000, 0.1, 5.0
    N = L ** 3
    K = pa_inputs.couplings_gauss16(L, pa_inputs.coupling_seed(3, 0))
    bound = int(np.abs(K.astype(np.int64)).sum())          # |E16| <= sum |k|
    g = pam.Population(L, R, K, pa_inputs.population_seed(3, 0, 0), layout="bitpack64",
                       model="gauss16")
    prev = g.observables()
    steps = 0
    while prev["beta"] < bmax:
        b = g.choose_beta(eps, bmax)
        g.resample(b)
        g.sweep(b, 10)
        o = g.observables()
        assert 0 < o["R_tilde"] and abs(o["R_tilde"] - R) <= 16 * math.isqrt(R) + 256
        assert o["rho_t"] >= 1.0 - 1e-12 and o["sum_eta2"] >= o["R_tilde"]
        assert -bound <= o["E_min"] <= bound
        assert o["E_min"] / 16.0 <= o["mean_E"] + 1e-9
        assert 1 <= o["n_at_E_min"] <= o["R_tilde"]
        assert o["step"] == prev["step"] + 1 and o["beta"] > prev["beta"]
        if b < bmax:
            assert o["eps_expected"] <= eps + 1e-12
        steps += 1
        prev = o
    say("gauss anneal steps", steps, prev)
    assert prev["beta"] == bmax and 50 < steps < 5000
    s, u, f = g.export_state()
    E = u.view(np.int32)
    assert np.all(np.diff(f.astype(np.int64)) >= 0)
    idx = np.sort(np.random.default_rng(5).choice(s.shape[0], 512, replace=False))
    np.testing.assert_array_equal(E[idx], props.energy16(L, K, s[idx]))
    assert prev["mean_E"] == E.astype(np.int64).sum() / E.size / 16.0
    assert prev["E_min"] == E.min() and prev["n_at_E_min"] == int(np.count_nonzero(E == E.min()))
    # the annealed population sits far below the beta = 0 energy scale
    assert prev["mean_E"] < -1.5 * N
    g.close()


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("L,R", [(4, 500), (12, 130), (14, 100), (16, 70)])
def test_sweep_parity_other_sizes(pam, layout, L, R):
    """Sweeps and a resampling step at the smallest and the two largest lattices
    (a ragged last tile in each)."""
    say("gauss sweep sizes", layout, L, R)
    K, g, o = pair(pam, L, R, 900 + L, layout, 40 + L)
    g.sweep(0.6, 2)
    o.sweep(0.6, 2)
    assert_state(g, o, f"L={L} swept")
    g.resample(0.7)
    o.resample(0.7)
    g.sweep(0.7, 3)
    o.sweep(0.7, 3)
    compare_obs(g.observables(), o.observables(), 1)
    assert_state(g, o, f"L={L} resampled and swept")
    g.close()


def test_capacity_overflow_keeps_population(pam):
    """With capacity R, a resampling step soon needs more slots: the call fails
    with PA_ECAPACITY and leaves the population as it was."""
    L, R = 4, 256
    K = pa_inputs.couplings_gauss16(L, 8)
    g = pam.Population(L, R, K, 5, capacity=R, layout="int8", model="gauss16")
    g.sweep(0.5, 2)
    before = g.export_state()
    failed = False
    for beta in np.linspace(0.5, 5.0, 40)[1:]:
        try:
            g.resample(float(beta))
        except pam.PAError as e:
            assert e.status == pam.PA_ECAPACITY
            failed = True
            break
        g.sweep(float(beta), 1)
        before = g.export_state()
    assert failed
    after = g.export_state()
    for x, y in zip(before, after):
        np.testing.assert_array_equal(x, y)
    g.close()


def test_wide_energy_window_global_histogram(pam):
    """A window wider than the LDS histogram (16384 levels): couplings all
    k = +127 and a population of 64 aligned replicas (E16 = -3 N 127) among
    random ones (E16 near 0) span about 2e5 levels, so the window histogram
    takes its global-atomic path.  Imported into both sides; one resampling
    step and sweeps bit-exact."""
    L, R = 8, 256
    N = L ** 3
    K = np.full(3 * N, 127, np.int8)
    rng = np.random.default_rng(11)
    spins = np.where(rng.random((R, N)) < 0.5, 1, -1).astype(np.int8)
    spins[:64] = 1
    fam = np.arange(R, dtype=np.uint32)
    o = oracle.GaussPopulation(L, K, R, 321)
    o.spins = spins.reshape(-1).copy()
    o.U = oracle.g_energy(L, K, o.spins)
    o.fam = fam.copy()
    lo, hi = o.window()
    assert hi - lo + 1 > 16384 and lo == -3 * N * 127
    g = pam.Population(L, R, K, 321, layout="bitpack64", model="gauss16")
    g.import_state(spins, fam, 0, 0, 0.0, 0.0)
    assert_state(g, o, "imported wide window")
    g.resample(2e-4)
    o.resample(2e-4)
    c, off = g.export_counts()
    np.testing.assert_array_equal(c, o.last["n"])
    np.testing.assert_array_equal(off.astype(np.uint64), o.last["offsets"])
    g.sweep(2e-4, 2)
    o.sweep(2e-4, 2)
    compare_obs(g.observables(), o.observables(), 1)
    assert_state(g, o, "wide window after a step")
    g.close()
