"""GPU: the batch engine (one captured graph per temperature step, replayed)
against the same instances run one call at a time.

Every population of a batch draws exactly the random numbers it draws alone,
and the device FP64 table repeats the host table's arithmetic, so every
per-step scalar (beta F, <E>, rho_t, ln Q, culling fraction, sizes, E_min),
every overlap histogram and the final states must be bit-identical.  The
single-instance path is itself bit-exact against the oracle
(test_gpu_parity.py), which closes the loop to the paper's algorithm
(Amey & Machta, arXiv:1711.02146, Sec. II).
"""
import numpy as np
import pytest

import oracle
import pa_inputs

pytestmark = pytest.mark.gpu

FIELDS = ("beta", "dbeta", "lnQ", "beta_F", "mean_E", "rho_t", "eps_expected", "R_tilde",
          "n_culled", "E_min", "step", "sum_eta2", "sweeps_done", "n_at_E_min")


@pytest.fixture(scope="module")
def pam():
    import torch

    assert torch.cuda.is_available()
    import paper_1711_02146_amd as m

    m.lib()
    return m


def make_instances(spec):
    """spec: list of (L, R, layout, instance id); two populations each, same couplings."""
    out = []
    for (L, R, layout, inst) in spec:
        J = pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(4, inst))
        out.append((L, R, layout, J, pa_inputs.population_seed(4, inst, 0),
                    pa_inputs.population_seed(4, inst, 1)))
    return out


def run_single(pam, insts, betas, n_sweeps):
    """Eager per-instance run: per step obs of every population, q hist per pair."""
    pops = []
    for (L, R, layout, J, sa, sb) in insts:
        pops.append(pam.Population(L, R, J, sa, layout=layout))
        pops.append(pam.Population(L, R, J, sb, layout=layout))
    obs, qs = [], []
    for k in range(1, len(betas)):
        row = []
        for p in pops:
            p.resample(betas[k])
            p.sweep(betas[k], n_sweeps)
            row.append(p.observables())
        obs.append(row)
        qs.append([pam.overlap_hist(pops[2 * i], pops[2 * i + 1]) for i in range(len(insts))])
    states = [p.export_state() for p in pops]
    for p in pops:
        p.close()
    return obs, qs, states


def run_batch(pam, insts, betas, n_sweeps, steps_per_run=None):
    import torch

    stream = torch.cuda.Stream()
    pops = []
    for (L, R, layout, J, sa, sb) in insts:
        pops.append(pam.Population(L, R, J, sa, layout=layout, stream=stream))
        pops.append(pam.Population(L, R, J, sb, layout=layout, stream=stream))
    pairs = [(2 * i, 2 * i + 1) for i in range(len(insts))]
    b = pam.Batch(pops, betas, n_sweeps, pairs=pairs)
    n = len(betas) - 1
    if steps_per_run:
        done = 0
        while done < n:
            k = min(steps_per_run, n - done)
            b.run(k)
            done += k
    else:
        b.run()
    recs, q, status = b.results()
    states = [p.export_state() for p in pops]
    b.close()
    for p in pops:
        p.close()
    return recs, q, status, states


def test_batch_matches_single_calls(pam):
    # mixed sizes and layouts; ragged R (not multiples of 64)
    spec = [(4, 700, "int8", 0), (6, 1000, "int8", 1), (8, 1500, "bitpack64", 2),
            (10, 900, "bitpack64", 3), (4, 333, "bitpack64", 4), (8, 2050, "int8", 5)]
    insts = make_instances(spec)
    betas = oracle.linear_schedule(5.0, 21)
    n_sweeps = 10
    obs_s, q_s, st_s = run_single(pam, insts, betas, n_sweeps)
    obs_b, q_b, status, st_b = run_batch(pam, insts, betas, n_sweeps, steps_per_run=7)
    assert np.all(status == 0)
    assert len(obs_b) == len(betas) - 1
    for k, (rs, rb) in enumerate(zip(obs_s, obs_b)):
        for p, (a, b) in enumerate(zip(rs, rb)):
            for f in FIELDS:
                assert a[f] == b[f], (k, p, f, a[f], b[f])
        for i in range(len(insts)):
            np.testing.assert_array_equal(q_s[k][i], q_b[k][i], err_msg=f"q step {k} pair {i}")
    for (s1, u1, f1), (s2, u2, f2) in zip(st_s, st_b):
        np.testing.assert_array_equal(s1, s2)
        np.testing.assert_array_equal(u1, u2)
        np.testing.assert_array_equal(f1, f2)


def test_batch_against_oracle_small(pam):
    """One instance (two populations) through the batch, checked against the oracle."""
    import torch

    L, R = 6, 800
    J = pa_inputs.couplings_pm(L, 77)
    betas = oracle.linear_schedule(3.0, 13)
    stream = torch.cuda.Stream()
    g = [pam.Population(L, R, J, s, layout="bitpack64", stream=stream) for s in (11, 12)]
    o = [oracle.Population(L, J, R, s) for s in (11, 12)]
    b = pam.Batch(g, betas, 10, pairs=[(0, 1)])
    b.run()
    recs, q, status = b.results()
    assert np.all(status == 0)
    for k in range(1, len(betas)):
        for p in o:
            p.resample(betas[k])
            p.sweep(betas[k], 10)
        ro = [p.observables() for p in o]
        qo, _ = oracle.overlap_hist(L ** 3, o[0].spins, o[1].spins)
        np.testing.assert_array_equal(q[k - 1][0], qo)
        for i in range(2):
            rb = recs[k - 1][i]
            assert rb["beta_F"] == ro[i].beta_F and rb["mean_E"] == ro[i].mean_E
            assert rb["rho_t"] == ro[i].rho_t and rb["R_tilde"] == ro[i].R_tilde
            assert rb["E_min"] == ro[i].E_min and rb["lnQ"] == ro[i].lnQ
    s, u, f = g[0].export_state()
    np.testing.assert_array_equal(s.reshape(-1), o[0].spins)
    # the instances are their own again: one more step on each side
    g[0].resample(3.25)
    g[0].sweep(3.25, 5)
    o[0].resample(3.25)
    o[0].sweep(3.25, 5)
    s, u, f = g[0].export_state()
    np.testing.assert_array_equal(s.reshape(-1), o[0].spins)
    np.testing.assert_array_equal(f, o[0].fam)
    b.close()
    for x in g:
        x.close()


def test_batch_capacity_overflow_stops_that_population(pam):
    import torch

    L, R = 4, 256
    J = pa_inputs.couplings_pm(L, 8)
    betas = list(np.linspace(0.0, 5.0, 41))
    stream = torch.cuda.Stream()
    tight = pam.Population(L, R, J, 5, capacity=R, layout="int8", stream=stream)
    roomy = pam.Population(L, R, J, 6, layout="int8", stream=stream)
    b = pam.Batch([tight, roomy], betas, 1)
    b.run()
    recs, q, status = b.results()
    assert status[0] == pam.PA_ECAPACITY and status[1] == 0
    k_fail = next(k for k in range(len(recs)) if recs[k][0]["step"] == 0)
    assert k_fail >= 1
    # the same population run alone fails at the same step and holds the same state
    ref = pam.Population(L, R, J, 5, capacity=R, layout="int8")
    for k in range(1, len(betas)):
        try:
            ref.resample(betas[k])
        except pam.PAError as e:
            assert e.status == pam.PA_ECAPACITY
            assert k == k_fail + 1
            break
        ref.sweep(betas[k], 1)
        assert ref.observables()["beta_F"] == recs[k - 1][0]["beta_F"]
    for x, y in zip(ref.export_state(), tight.export_state()):
        np.testing.assert_array_equal(x, y)
    b.close()
    for x in (tight, roomy, ref):
        x.close()
