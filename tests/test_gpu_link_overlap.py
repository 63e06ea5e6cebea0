"""GPU parity for the link-overlap histogram (Sec. II.A link overlap q_l over
the 3N bonds, two populations of one disorder sample, slot i against slot i).

The HIP library's counts of D = 0..3N (q_l = 1 - 2 D / 3N) must equal the
oracle's, computed from the oracle's own populations run in lockstep on the
same seeds: bit-exact, every step, both spin layouts and both coupling models,
ragged and unequal population sizes, L = 4 to 16.  Amey & Machta,
arXiv:1711.02146, Sec. II.A.
"""
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

    assert torch.cuda.is_available()
    import paper_1711_02146_amd as m

    m.lib()
    return m


def _check(pam, L, ga, gb, oa, ob, what):
    h = pam.link_overlap_hist(ga, gb)
    ho, _ = oracle.link_overlap(L, oa.spins, ob.spins)
    assert h.size == 3 * L ** 3 + 1
    np.testing.assert_array_equal(h, ho, err_msg="link overlap " + what)
    assert int(h.sum()) == min(oa.R_tilde, ob.R_tilde), what
    return h


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
def test_link_overlap_pm_every_step(pam, layout):
    """+-J, L=8, R=3000 (ragged last tile), two populations through 12 steps."""
    L, R = 8, 3000
    J = pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(5, 0))
    sa, sb = pa_inputs.population_seed(5, 0, 0), pa_inputs.population_seed(5, 0, 1)
    say("link overlap pm", layout, L, R)
    ga = pam.Population(L, R, J, sa, layout=layout)
    gb = pam.Population(L, R, J, sb, layout=layout)
    oa = oracle.Population(L, J, R, sa)
    ob = oracle.Population(L, J, R, sb)
    _check(pam, L, ga, gb, oa, ob, "beta 0")
    betas = oracle.linear_schedule(3.0, 13)
    ql = []
    for k in range(1, 13):
        for g, o in ((ga, oa), (gb, ob)):
            g.resample(betas[k])
            o.resample(betas[k])
            g.sweep(betas[k], 5)
            o.sweep(betas[k], 5)
        h = _check(pam, L, ga, gb, oa, ob, f"step {k}")
        D = np.arange(h.size)
        ql.append(float((h * (1.0 - 2.0 * D / (3 * L ** 3))).sum() / h.sum()))
    # <q_l> rises from ~0 (independent random spins) as the populations order
    assert abs(ql[0]) < 0.1 and ql[-1] > 0.3
    ga.close()
    gb.close()


def test_link_overlap_gauss16_steps(pam):
    """Quantised Gaussian couplings, L=6, R=1000, 8 steps."""
    L, R = 6, 1000
    K = pa_inputs.couplings_gauss16(L, 31)
    say("link overlap gauss16", L, R)
    ga = pam.Population(L, R, K, 11, model="gauss16")
    gb = pam.Population(L, R, K, 12, model="gauss16")
    oa = oracle.GaussPopulation(L, K, R, 11)
    ob = oracle.GaussPopulation(L, K, R, 12)
    betas = oracle.linear_schedule(2.0, 9)
    for k in range(1, 9):
        for g, o in ((ga, oa), (gb, ob)):
            g.resample(betas[k])
            o.resample(betas[k])
            g.sweep(betas[k], 4)
            o.sweep(betas[k], 4)
        _check(pam, L, ga, gb, oa, ob, f"step {k}")
    ga.close()
    gb.close()


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("L,Ra,Rb", [(4, 100, 77), (10, 333, 500), (12, 64, 65), (16, 130, 200)])
def test_link_overlap_sizes(pam, layout, L, Ra, Rb):
    """Unequal sizes (the first min(R~a, R~b) pairs), L up to the maximum 16."""
    J = pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(6, L))
    say("link overlap sizes", layout, L, Ra, Rb)
    ga = pam.Population(L, Ra, J, 7, layout=layout)
    gb = pam.Population(L, Rb, J, 8, layout=layout)
    oa = oracle.Population(L, J, Ra, 7)
    ob = oracle.Population(L, J, Rb, 8)
    _check(pam, L, ga, gb, oa, ob, "beta 0")
    for b in (0.4, 0.9):
        for g, o in ((ga, oa), (gb, ob)):
            g.resample(b)
            o.resample(b)
            g.sweep(b, 2)
            o.sweep(b, 2)
        _check(pam, L, ga, gb, oa, ob, f"beta {b}")
    # the pair order is (a, b): swapping the populations gives the same counts
    np.testing.assert_array_equal(pam.link_overlap_hist(gb, ga), pam.link_overlap_hist(ga, gb))
    ga.close()
    gb.close()


def test_link_overlap_rejects_bad_arguments(pam):
    L = 4
    J = pa_inputs.couplings_pm(L, 3)
    a = pam.Population(L, 100, J, 1)
    b = pam.Population(L, 100, J, 2)
    c = pam.Population(6, 100, pa_inputs.couplings_pm(6, 3), 3)
    d = pam.Population(L, 100, J, 4, layout="int8")
    for x, y, nb in ((a, a, 3 * L ** 3 + 1), (a, b, 65), (a, b, 3 * L ** 3), (a, c, 3 * L ** 3 + 1),
                     (a, d, 3 * L ** 3 + 1)):
        with pytest.raises(pam.PAError) as e:
            pam.pa_link_overlap_hist(x.handle, y.handle, nb)
        assert e.value.status == pam.PA_EINVAL
    # the instances are still usable afterwards
    assert int(pam.link_overlap_hist(a, b).sum()) == 100
    for p in (a, b, c, d):
        p.close()
