"""Full-size parity, every step: the HIP library against per-step digests of
the CPU oracle's run of the same workload (tests/golden/fullsize_*.json,
written by tests/golden/make_fullsize_digests.py, which calls only the oracle).

C3 (L = 10, R = 5e5, bit-packed, constant culling eps = 0.1, N_S = 10): the
first 25 steps, in both sweep launch forms (4 and 8 waves per tile; the
benchmark's autotuner may time either).  C2 (L = 8, R = 1e5, int8, two
populations, linear schedule of 201 temperatures): the first 10 steps of both
populations and their overlap histograms.

Per step: the chosen beta, the copy counts and offsets of the resampling
step, the spins, energy words and family labels after the sweeps (bit-exact,
through their digests), the integer scalars and the FP64 scalars (beta F, <E>,
rho_t, ln Q, eps, dbeta) exactly: the digests store the oracle's doubles in
hexadecimal, and both sides form them by the same IEEE operations (Sec. II
loop; Eqs. 1-2, 9; Sec. III.A, III.C).
"""
import os
import sys

import numpy as np
import pytest

import pa_inputs

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import fullsize as fs  # noqa: E402

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
    return m


def check_step(g, want, obs, where):
    for k in fs.FLOATS:
        assert obs[k] == float.fromhex(want[k]), (where, k, obs[k].hex(), want[k])
    for k in fs.INTS:
        assert int(obs[k]) == want[k], (where, k, obs[k], want[k])
    assert obs["step"] == want["k"], where


def check_state(g, want, counts, offsets, where):
    assert fs.u32_digest(counts) == want["counts"], ("counts", where)
    assert fs.u32_digest(offsets) == want["offsets"], ("offsets", where)
    s, u, f = g.export_state()
    assert s.shape[0] == want["R_tilde"], where
    assert fs.u32_digest(f) == want["family"], ("family", where)
    assert fs.u32_digest(u) == want["U"], ("U", where)
    assert fs.spins_digest(s, s.shape[0], s.shape[1]) == want["spins"], ("spins", where)


@pytest.mark.parametrize("split", [4, 8])
def test_c3_first_steps_every_bit(pam, split):
    gold = fs.load("C3")
    w = gold["workload"]
    L, R = w["L"], w["R"]
    J = pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(w["config"], 0))
    pam.pa_autotune_reset()
    try:
        for tiles in (4096, 8192):  # the size classes R~ passes through (7.8e3 tiles)
            pam.pa_autotune_set(L, 64 * tiles, split, layout="bitpack64")
        g = pam.Population(L, R, J, gold["seed"], layout="bitpack64")
        for want in gold["steps"]:
            k = want["k"]
            say("C3 split", split, "step", k)
            b = g.choose_beta(w["eps"], w["beta_max"])
            assert b == float.fromhex(want["beta"]), (k, b, want["beta"])
            g.resample(b)
            counts, offsets = g.export_counts()
            g.sweep(b, w["n_sweeps"])
            check_step(g, want, g.observables(), f"C3 step {k}")
            check_state(g, want, counts, offsets, f"C3 step {k}")
        g.close()
    finally:
        pam.pa_autotune_reset()


def test_c2_first_steps_every_bit(pam):
    gold = fs.load("C2")
    w = gold["workload"]
    L, R = w["L"], w["R"]
    J = pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(w["config"], 0))
    pops = [pam.Population(L, R, J, s, layout="int8") for s in gold["seeds"]]
    betas = pam.linear_schedule(w["beta_max"], w["n_temps"])
    for want in gold["steps"]:
        k = want["pops"][0]["k"]
        say("C2 step", k)
        for g, wp in zip(pops, want["pops"]):
            g.resample(betas[k])
            counts, offsets = g.export_counts()
            g.sweep(betas[k], w["n_sweeps"])
            check_step(g, wp, g.observables(), f"C2 step {k}")
            check_state(g, wp, counts, offsets, f"C2 step {k}")
        q = pam.overlap_hist(pops[0], pops[1])
        np.testing.assert_array_equal(q, np.array(want["q"], np.uint64), err_msg=f"q step {k}")
    for g in pops:
        g.close()
