"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bit-exact on spins, energies U, family labels, copy counts and offsets; the
FP64 scalars (beta F, <E>, rho_t, the adaptive beta) must agree to 1e-12
relative -- they are computed from identical integers by identical
operation orders, so in practice they are equal.

Method: Amey & Machta, arXiv:1711.02146 (Sec. II loop, Eqs. 1-2, Eq. 9,
Sec. III.A, Sec. III.C).
"""
import math
import sys

import numpy as np
import pytest

import oracle
import pa_inputs

pytestmark = pytest.mark.gpu

REL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pam():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1711_02146_amd as m

    m.lib()
    return m


def pair(pam, L, R, seed, layout, cseed, capacity=0):
    J = pa_inputs.couplings_pm(L, cseed)
    g = pam.Population(L, R, J, seed, capacity=capacity, layout=layout)
    o = oracle.Population(L, J, R, seed, capacity=capacity or None)
    return J, g, o


def assert_state(g, o, what=""):
    s, u, f = g.export_state()
    assert s.shape[0] == o.R_tilde, what
    np.testing.assert_array_equal(s.reshape(-1), o.spins, err_msg="spins " + what)
    np.testing.assert_array_equal(u.astype(np.int32), o.U, err_msg="U " + what)
    np.testing.assert_array_equal(f, o.fam, err_msg="family " + what)


def close(a, b):
    return a == b or abs(a - b) <= REL * max(abs(a), abs(b))


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("L,R", [(4, 1000), (6, 77), (8, 129), (10, 333), (12, 64), (16, 65)])
def test_init_parity(pam, layout, L, R):
    say("init", layout, L, R)
    J, g, o = pair(pam, L, R, 0x5EED0000 + L, layout, 17 + L)
    assert_state(g, o, f"init L={L} R={R}")
    g.close()


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("beta", [0.0, 0.3, 1.0, 5.0])
def test_sweep_parity(pam, layout, beta):
    L, R = 8, 300
    say("sweep", layout, beta)
    J, g, o = pair(pam, L, R, 1234, layout, 5)
    g.sweep(beta, 3)
    o.sweep(beta, 3)
    assert_state(g, o, f"after 3 sweeps at beta={beta}")
    g.sweep(beta, 2)
    o.sweep(beta, 2)
    assert_state(g, o, f"after 5 sweeps at beta={beta}")
    g.close()


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("L,R", [(4, 140000), (6, 140000), (4, 131071), (6, 5000)])
def test_sweep_forms_parity(pam, layout, L, R):
    """Both sweep forms under the built-in rule: four waves per tile (the large
    launches at L = 4 and 6) and eight (the small one), each bit-exact against
    the oracle, through two resampling steps (gather fused into the sweep) at
    beta 0.4, 0.8."""
    say("sweep forms", layout, L, R)
    J, g, o = pair(pam, L, R, 4321 + R, layout, 9 + L)
    for b in (0.4, 0.8):
        g.resample(b)
        o.resample(b)
        g.sweep(b, 2)
        o.sweep(b, 2)
        assert_state(g, o, f"L={L} R={R} after the step to beta={b}")
    g.close()


def _compare_step(g, o, k):
    c, off = g.export_counts()
    np.testing.assert_array_equal(c, o.last["n"], err_msg=f"counts step {k}")
    np.testing.assert_array_equal(off.astype(np.uint64), o.last["offsets"],
                                  err_msg=f"offsets step {k}")


def _compare_obs(go, rec, k):
    assert go["R_tilde"] == rec.R_tilde, k
    assert go["E_min"] == rec.E_min, k
    assert go["n_at_E_min"] == rec.n_at_E_min, k
    assert go["sum_eta2"] == rec.sum_eta2, k
    assert go["step"] == rec.k
    for key in ("beta", "beta_F", "mean_E", "rho_t", "lnQ", "eps_expected", "dbeta"):
        assert close(go[key], getattr(rec, key)), (k, key, go[key], getattr(rec, key))
    assert go["n_culled"] == rec.n_culled, k


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("L,R,beta", [(4, 20000, 5.0), (6, 5000, 1.5), (10, 70000, 0.3)])
def test_one_large_step_concentrates_copies(pam, layout, L, R, beta):
    """One resampling step from beta = 0 straight to beta: a few low-energy
    replicas take most of the new population (thousands of copies each, more
    than one block of old slots holds), and the copy map must still be exact."""
    say("large step", layout, L, R, beta)
    J, g, o = pair(pam, L, R, 0x5EED0700 + L, layout, 70 + L)
    g.resample(beta)
    o.resample(beta)
    _compare_step(g, o, 1)
    assert int(o.last["n"].max()) > 1024
    g.sweep(beta, 2)
    o.sweep(beta, 2)
    assert_state(g, o, f"after the step to beta={beta}")
    _compare_obs(g.observables(), o.observables(), 1)
    g.close()


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
def test_linear_run_l4_every_step(pam, layout):
    """Plain PA at L=4, R=1000, N_T=51 to beta=5, N_S=10: every step bit-exact."""
    L, R = 4, 1000
    J, g, o = pair(pam, L, R, pa_inputs.population_seed(1, 0, 0), layout,
                   pa_inputs.coupling_seed(1, 0))
    betas = oracle.linear_schedule(5.0, 51)
    for k in range(1, 51):
        g.resample(betas[k])
        o.resample(betas[k])
        _compare_step(g, o, k)
        g.sweep(betas[k], 10)
        o.sweep(betas[k], 10)
        rec = o.observables()
        _compare_obs(g.observables(), rec, k)
        if k % 5 == 0 or k == 50:
            assert_state(g, o, f"step {k}")
    say("L4 final", layout, rec)
    g.close()


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
def test_two_population_overlap_l8(pam, layout):
    """Two populations, same couplings, different seeds: q histogram per beta."""
    L, R = 8, 3000
    J = pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(2, 0))
    sa, sb = pa_inputs.population_seed(2, 0, 0), pa_inputs.population_seed(2, 0, 1)
    ga = pam.Population(L, R, J, sa, layout=layout)
    gb = pam.Population(L, R, J, sb, layout=layout)
    oa = oracle.Population(L, J, R, sa)
    ob = oracle.Population(L, J, R, sb)
    betas = oracle.linear_schedule(5.0, 21)
    h0 = pam.overlap_hist(ga, gb)
    q0, _ = oracle.overlap_hist(L ** 3, oa.spins, ob.spins)
    np.testing.assert_array_equal(h0, q0)
    for k in range(1, 21):
        for g, o in ((ga, oa), (gb, ob)):
            g.resample(betas[k])
            o.resample(betas[k])
            g.sweep(betas[k], 10)
            o.sweep(betas[k], 10)
        h = pam.overlap_hist(ga, gb)
        q, _ = oracle.overlap_hist(L ** 3, oa.spins, ob.spins)
        np.testing.assert_array_equal(h, q, err_msg=f"q histogram step {k}")
        assert int(h.sum()) == min(oa.R_tilde, ob.R_tilde)
    assert_state(ga, oa, "pop A final")
    assert_state(gb, ob, "pop B final")
    ga.close()
    gb.close()


def test_adaptive_prefix_l10_bitpack(pam):
    """Constant culling eps = 0.1 (dbeta solved on a bracket), bit-packed L=10."""
    L, R = 10, 2000
    J, g, o = pair(pam, L, R, pa_inputs.population_seed(3, 0, 0), "bitpack64",
                   pa_inputs.coupling_seed(3, 0))
    for k in range(1, 16):
        bg = g.choose_beta(0.1, 5.0)
        bo = o.choose_beta(0.1, 5.0)
        assert bg == bo, (k, bg, bo)
        g.resample(bg)
        o.resample(bo)
        _compare_step(g, o, k)
        g.sweep(bg, 10)
        o.sweep(bo, 10)
        _compare_obs(g.observables(), o.observables(), k)
    assert_state(g, o, "adaptive prefix")
    g.close()


def test_layouts_agree(pam):
    L, R = 6, 500
    J = pa_inputs.couplings_pm(L, 3)
    a = pam.Population(L, R, J, 99, layout="int8")
    b = pam.Population(L, R, J, 99, layout="bitpack64")
    for beta in (0.2, 0.6, 1.0):
        for p in (a, b):
            p.resample(beta)
            p.sweep(beta, 4)
    sa, ua, fa = a.export_state()
    sb, ub, fb = b.export_state()
    np.testing.assert_array_equal(sa, sb)
    np.testing.assert_array_equal(ua, ub)
    np.testing.assert_array_equal(fa, fb)
    a.close()
    b.close()


def test_capacity_overflow_keeps_population(pam):
    L, R = 4, 256
    J = pa_inputs.couplings_pm(L, 8)
    g = pam.Population(L, R, J, 5, capacity=R, layout="int8")
    g.sweep(0.5, 2)
    before = g.export_state()
    # a large step concentrates copies on the lowest levels; with capacity R
    # some step soon overflows (R~' > R): the call must fail and change nothing
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


def test_import_state_roundtrip(pam):
    """A state built by the oracle, imported, swept on both sides."""
    L, R = 8, 200
    J = pa_inputs.couplings_pm(L, 12)
    o = oracle.Population(L, J, R, seed=4242)
    o.sweep(0.7, 3)
    g = pam.Population(L, R, J, 4242, layout="bitpack64")
    g.import_state(o.spins.reshape(R, -1), o.fam, o.t, o.k, o.beta, o.sum_lnQ)
    assert_state(g, o, "imported")
    g.sweep(0.9, 2)
    o.sweep(0.9, 2)
    assert_state(g, o, "imported + swept")
    g.close()


def test_errors(pam):
    J = pa_inputs.couplings_pm(4, 1)
    with pytest.raises(pam.PAError):
        pam.Population(5, 100, pa_inputs.couplings_pm(5, 1), 1)  # odd L
    with pytest.raises(pam.PAError):
        pam.Population(4, 0, J, 1)
    g = pam.Population(4, 100, J, 1, layout="int8")
    with pytest.raises(pam.PAError) as e:
        g.choose_beta(0.1, 0.0)  # beta_max must exceed beta
    assert e.value.status == pam.PA_EINVAL
    g.close()


# ---------------------------------------------------------------------------
# full sizes, sampled: the oracle builds its own population (init is cheap),
# computes the whole first resampling step, and sweeps sampled new slots one
# by one from its own gathered spins.
# ---------------------------------------------------------------------------
def _first_step_sampled(pam, L, R, layout, seed, cseed, adaptive, n_samples=192):
    J = pa_inputs.couplings_pm(L, cseed)
    N = L ** 3
    say("full-size", L, R, layout)
    g = pam.Population(L, R, J, seed, layout=layout)
    o = oracle.Population(L, J, R, seed)
    s, u, f = g.export_state()
    np.testing.assert_array_equal(s.reshape(-1), o.spins)
    np.testing.assert_array_equal(u.astype(np.int32), o.U)
    del s
    if adaptive:
        bg = g.choose_beta(0.1, 5.0)
        bo = o.choose_beta(0.1, 5.0)
        assert bg == bo
    else:
        bg = bo = 5.0 / 200
    g.resample(bg)
    h = o.histogram()
    fl, T, tau, lnQ, jmin = oracle.table(h, N, R, R, bo)
    n = oracle.copy_counts(o.U, fl, T, o.seed, 1)
    c, off = g.export_counts()
    np.testing.assert_array_equal(c, n)
    excl = np.concatenate([[0], np.cumsum(n.astype(np.int64))[:-1]])
    np.testing.assert_array_equal(off.astype(np.int64), excl)
    Rn = int(n.sum())
    src = np.repeat(np.arange(R, dtype=np.int64), n)
    g.sweep(bg, 10)
    s2, u2, f2 = g.export_state()
    assert s2.shape[0] == Rn
    np.testing.assert_array_equal(f2, o.fam[src])
    rng = np.random.default_rng(L * 1000 + R)
    pick = np.unique(np.concatenate([rng.integers(0, Rn, n_samples), [0, Rn - 1]]))
    sp = o.spins.reshape(R, N)[src[pick]].copy()
    U = o.U[src[pick]].copy()
    oracle.sweep_slots(L, J, sp, U, pick.astype(np.uint32), o.seed, bo, 0, 10)
    np.testing.assert_array_equal(s2[pick], sp)
    np.testing.assert_array_equal(u2[pick].astype(np.int32), U)
    # properties at any size: U matches the exported spins; labels sorted
    Uall = oracle.energy(L, J, s2)
    np.testing.assert_array_equal(u2.astype(np.int32), Uall)
    assert np.all(np.diff(f2.astype(np.int64)) >= 0)
    obs = g.observables()
    assert obs["R_tilde"] == Rn
    g.close()


def test_full_size_l10_r500k_bitpack_adaptive(pam):
    _first_step_sampled(pam, 10, 500000, "bitpack64", pa_inputs.population_seed(3, 0, 0),
                        pa_inputs.coupling_seed(3, 0), adaptive=True)


def test_full_size_l8_r100k_int8_linear(pam):
    _first_step_sampled(pam, 8, 100000, "int8", pa_inputs.population_seed(2, 0, 0),
                        pa_inputs.coupling_seed(2, 0), adaptive=False)


@pytest.mark.parametrize("split", [4, 8])
@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("L,R", [(12, 130), (14, 100), (16, 70)])
def test_sweep_parity_large_lattices(pam, layout, L, R, split):
    """The largest lattices (lower occupancy): sweeps, a resampling step and
    more sweeps, each with a ragged last tile, in both sweep forms (4 and 8
    waves per tile, pinned for every size class these populations pass through;
    each form has its own plane-group size at L = 14)."""
    say("large lattice", layout, L, R, split)
    pam.pa_autotune_reset()
    try:
        for tiles in (1, 2, 4, 8):
            pam.pa_autotune_set(L, 64 * tiles, split, layout=layout)
        _large_lattice_steps(pam, layout, L, R)
    finally:
        pam.pa_autotune_reset()


def _large_lattice_steps(pam, layout, L, R):
    J, g, o = pair(pam, L, R, 700 + L, layout, 60 + L)
    g.sweep(0.5, 2)
    o.sweep(0.5, 2)
    assert_state(g, o, f"L={L} swept")
    g.resample(0.6)
    o.resample(0.6)
    _compare_step(g, o, 1)
    g.sweep(0.6, 3)
    o.sweep(0.6, 3)
    _compare_obs(g.observables(), o.observables(), 1)
    assert_state(g, o, f"L={L} resampled and swept")
    g.close()


@pytest.mark.parametrize("split", [4, 8])
def test_full_size_l10_r500k_bitpack_both_forms(pam, split):
    """The full-size first step in both launch configurations the benchmark
    may time: its autotuner picks 4 or 8 waves per tile for this shape, by
    device and run, so each form is pinned here in turn."""
    L, R = 10, 500000
    pam.pa_autotune_reset()
    try:
        pam.pa_autotune_set(L, R, split, layout="bitpack64")
        _first_step_sampled(pam, L, R, "bitpack64", pa_inputs.population_seed(3, 0, 0),
                            pa_inputs.coupling_seed(3, 0), adaptive=True)
    finally:
        pam.pa_autotune_reset()
