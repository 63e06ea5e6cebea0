"""GPU parity of the real Gaussian-coupling model (Sec. II.A couplings as real
numbers on the grid 2^-32) against the CPU oracle, bit for bit: spins, energies
(exact FP64), family labels, copy counts and offsets, and the FP64 scalars of
every step (beta of the constant-culling bisection, ln Q, eps, beta F, <E>,
rho_t) compared with ==, since both sides compute them by the same sequence
of IEEE operations (Sec. II loop, Eqs. 1-2, 9; Sec. III.A, III.C)."""
import math
import sys

import numpy as np
import pytest

import oracle
import pa_inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pam():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1711_02146_amd as m

    m.lib()
    yield m
    m.pa_autotune_reset()


def pair(pam, L, R, cseed, seed, layout="bitpack64", **kw):
    J = pa_inputs.couplings_gauss(L, cseed)
    g = pam.Population(L, R, J, seed, layout=layout, model="gauss", **kw)
    o = oracle.GaussRealPopulation(L, J, R, seed)
    return J, g, o


def same_state(g, o, where=""):
    s, E, f = g.export_state()
    assert s.shape[0] == o.R_tilde, where
    np.testing.assert_array_equal(s.reshape(-1), o.spins, err_msg=f"spins {where}")
    np.testing.assert_array_equal(E, o.U[: o.R_tilde], err_msg=f"energies {where}")
    np.testing.assert_array_equal(f, o.fam[: o.R_tilde], err_msg=f"families {where}")


def same_obs(obs, rec, where=""):
    for k in ("beta", "dbeta", "lnQ", "beta_F", "mean_E", "rho_t", "eps_expected"):
        assert obs[k] == getattr(rec, k), (where, k, obs[k], getattr(rec, k))
    for k in ("R_tilde", "n_culled", "sum_eta2", "n_at_E_min"):
        assert obs[k] == getattr(rec, k), (where, k, obs[k], getattr(rec, k))
    assert obs["E_lowest"] == rec.E_min, (where, obs["E_lowest"], rec.E_min)
    assert obs["step"] == rec.k, where


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("L,R", [(4, 1000), (6, 77), (8, 129), (12, 64), (16, 65)])
def test_init_energies_exact(pam, layout, L, R):
    say("init", layout, L, R)
    J, g, o = pair(pam, L, R, 100 + L, 7 + L, layout)
    same_state(g, o, "init")
    r = g.observables()
    assert r["E_lowest"] == float(o.U.min()) and r["E_min"] == 0
    assert r["mean_E"] == o.observables().mean_E
    g.close()


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("beta", [0.0, 0.3, 1.0, 5.0])
def test_sweep_parity(pam, layout, beta):
    L, R = 8, 300
    say("sweep", layout, beta)
    J, g, o = pair(pam, L, R, 21, 5, layout)
    for n in (1, 4):
        g.sweep(beta, n)
        o.sweep(beta, n)
        same_state(g, o, f"beta {beta} after {n}")
    g.close()


@pytest.mark.parametrize("split", [4, 8])
@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("L,R", [(10, 200), (14, 100), (16, 70), (6, 140000)])
def test_sweep_forms_and_lattices(pam, layout, L, R, split):
    """Both sweep forms (4 and 8 waves per tile) at the largest lattices and
    at a population of two thousand tiles, each with a ragged last tile."""
    say("forms", layout, L, R, split)
    pam.pa_autotune_reset()
    try:
        pam.pa_autotune_set(L, R, split, layout=layout, model="gauss")
        J, g, o = pair(pam, L, R, 31 + L, 9, layout)
        g.sweep(0.7, 2)
        o.sweep(0.7, 2)
        same_state(g, o, "sweeps")
        g.resample(0.9)
        o.resample(0.9)
        pam.pa_autotune_set(L, o.R_tilde, split, layout=layout, model="gauss")
        g.sweep(0.9, 1)
        o.sweep(0.9, 1)
        same_state(g, o, "after a step")
        g.close()
    finally:
        pam.pa_autotune_reset()


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
def test_linear_schedule_every_step(pam, layout):
    """Plain PA at L = 6, R = 3000, N_T = 31 to beta = 3, N_S = 5: every step's
    counts, offsets, state and scalars bit-exact."""
    L, R = 6, 3000
    say("linear", layout)
    J, g, o = pair(pam, L, R, 41, 11, layout)
    betas = oracle.linear_schedule(3.0, 31)
    for k in range(1, len(betas)):
        rs = g.resample(betas[k])
        o.resample(betas[k])
        c, off = g.export_counts()
        np.testing.assert_array_equal(c, o.last["n"], err_msg=f"counts {k}")
        np.testing.assert_array_equal(off, o.last["offsets"].astype(np.uint32),
                                      err_msg=f"offsets {k}")
        assert rs["lnQ"] == o.last["lnQ"] and rs["eps_expected"] == o.last["eps"], k
        g.sweep(betas[k], 5)
        o.sweep(betas[k], 5)
        same_obs(g.observables(), o.observables(), f"step {k}")
        same_state(g, o, f"step {k}")
    g.close()


def test_constant_culling_every_step(pam):
    """The bisection on the device: every beta equal to the oracle's, then the
    step and its scalars (L = 8, R = 4000, eps = 0.1, to beta = 2)."""
    L, R = 8, 4000
    J, g, o = pair(pam, L, R, 51, 13)
    k = 0
    while o.beta < 2.0:
        k += 1
        say("adaptive step", k)
        b = g.choose_beta(0.1, 2.0)
        bo = o.choose_beta(0.1, 2.0)
        assert b == bo, (k, b, bo)
        g.resample(b)
        o.resample(bo)
        g.sweep(b, 5)
        o.sweep(bo, 5)
        same_obs(g.observables(), o.observables(), f"step {k}")
        same_state(g, o, f"step {k}")
    assert k > 5 and g.observables()["beta"] == 2.0
    g.close()


def test_anneal_run_equals_the_oracle(pam):
    """pa_anneal_run (the separate calls, step by step, for this model) against
    the oracle's choose/resample/sweep loop."""
    L, R = 6, 5000
    J, g, o = pair(pam, L, R, 61, 17)
    recs = g.anneal_run(0.2, 3.0, 4, 1000)
    for k, r in enumerate(recs):
        b = o.choose_beta(0.2, 3.0)
        o.resample(b)
        o.sweep(b, 4)
        same_obs(r, o.observables(), f"run step {k + 1}")
    assert o.beta == 3.0
    same_state(g, o, "end")
    g.close()


def test_zero_step_overflow_and_impossible_target(pam):
    L, R = 6, 2000
    J, g, o = pair(pam, L, R, 71, 19)
    g.sweep(0.5, 3)
    o.sweep(0.5, 3)
    # dbeta = 0 (beta is still 0): every replica gets one copy
    r = g.resample(0.0)
    o.resample(0.0)
    assert r["lnQ"] == 0.0 and r["eps_expected"] == 0.0
    c, _ = g.export_counts()
    assert np.all(c == 1)
    g.sweep(0.0, 1)
    o.sweep(0.0, 1)
    same_state(g, o, "identity step")
    # the population is above R after a step: eps(0) > 0 = target is impossible
    b = g.choose_beta(0.3, 5.0)
    g.resample(b)
    o.resample(o.choose_beta(0.3, 5.0))
    g.sweep(b, 1)
    o.sweep(b, 1)
    if o.R_tilde > R:
        with pytest.raises(pam.PAError) as e:
            g.choose_beta(0.0, 5.0)
        assert e.value.status == pam.PA_ESCHEDULE
    same_state(g, o, "end")
    g.close()


def test_energy_check_and_checkpoint(pam):
    """The debug energy check passes on real runs; a checkpoint (spins,
    families, counters, sum ln Q) taken at step k and imported into a fresh
    instance continues bit-identically."""
    L, R = 6, 1500
    J = pa_inputs.couplings_gauss(L, 81)
    g = pam.Population(L, R, J, 23, model="gauss", flags=pam.PA_FLAG_CHECK_ENERGY)
    betas = oracle.linear_schedule(2.0, 21)
    for k in range(1, 8):
        g.resample(betas[k])
        g.sweep(betas[k], 3)
    s, E, f = g.export_state()
    r = g.observables()
    h = pam.Population(L, R, J, 23, model="gauss")
    h.import_state(s, f, r["sweeps_done"], r["step"], r["beta"], r["sum_lnQ"])
    s2, E2, f2 = h.export_state()
    np.testing.assert_array_equal(E2, E)
    for k in range(8, 21):
        for p in (g, h):
            p.resample(betas[k])
            p.sweep(betas[k], 3)
        assert g.observables() == h.observables(), k
    for x, y in zip(g.export_state(), h.export_state()):
        np.testing.assert_array_equal(x, y)
    g.close()
    h.close()


def test_couplings_rounded_to_the_grid(pam):
    """Couplings off the grid are rounded to the nearest multiple of 2^-32:
    the population equals one created from the rounded couplings."""
    L, R = 4, 500
    J = pa_inputs.couplings_gauss(L, 91)
    off = J + np.ldexp(0.3, -32) * np.where(np.arange(J.size) % 2 == 0, 1.0, -1.0)
    a = pam.Population(L, R, J, 3, model="gauss")
    b = pam.Population(L, R, off, 3, model="gauss")
    for p in (a, b):
        p.resample(0.4)
        p.sweep(0.4, 3)
    for x, y in zip(a.export_state(), b.export_state()):
        np.testing.assert_array_equal(x, y)
    a.close()
    b.close()


def test_capacity_overflow_at_the_same_step(pam):
    """Capacity exactly R: the first step whose copies exceed it fails on both
    sides alike (PA_ECAPACITY, the population untouched), the steps before it
    succeed alike."""
    L, R = 4, 700
    J = pa_inputs.couplings_gauss(L, 73)
    g = pam.Population(L, R, J, 29, model="gauss", capacity=R)
    o = oracle.GaussRealPopulation(L, J, R, 29, capacity=R)
    failed = False
    for k, b in enumerate(oracle.linear_schedule(4.0, 41)[1:], 1):
        try:
            o.resample(b)
        except OverflowError:
            with pytest.raises(pam.PAError) as e:
                g.resample(b)
            assert e.value.status == pam.PA_ECAPACITY, k
            same_state(g, o, f"after the overflow at step {k}")
            failed = True
            break
        g.resample(b)
        g.sweep(b, 2)
        o.sweep(b, 2)
        same_state(g, o, f"step {k}")
    assert failed
    g.close()


def test_draw_of_all_ones_takes_the_exact_threshold(pam):
    """The sweep decides with min(thr, 2^32 - 1) and reads the exact threshold
    only for the draw 2^32 - 1, where 2^32 (taken) and 2^32 - 1 (not taken)
    part.  At beta = 0 every threshold is 2^32, so the draw 2^32 - 1 that
    replica 58 gets at site 0 in the first sweep under this seed (pinned
    against rocRAND's Philox in test_philox_layout_pins.py) is taken like
    every other move: one sweep flips every spin, as in the oracle."""
    L, R, seed = 4, 64, 0x5EED0000000C56F4
    say("top draw", L, R, hex(seed))
    J, g, o = pair(pam, L, R, 0xC0DE0777, seed)
    start = o.spins.copy()
    g.sweep(0.0, 1)
    o.sweep(0.0, 1)
    same_state(g, o, "one sweep at beta = 0")
    np.testing.assert_array_equal(o.spins, -start)
    g.close()
