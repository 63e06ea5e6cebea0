"""GPU: continuous batching.  The stepper advances a changing set of resident
instances by one temperature step per call; each instance must end every step
exactly where the same calls made on it alone leave it (Sec. II loop of Amey &
Machta, arXiv:1711.02146: resample with Eqs. 1-2, sweeps, observables), and a
served request's results must not depend on the other requests in the mix.
"""
import numpy as np
import pytest

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


def linear(beta_max, n_temps):
    return [beta_max * k / (n_temps - 1) for k in range(n_temps)]


# (L, R, layout, n_temps, n_sweeps, join tick)
SPEC = [(4, 700, "int8", 9, 10, 0), (6, 1000, "bitpack64", 12, 5, 0), (8, 1500, "bitpack64", 7, 10, 2),
        (10, 900, "int8", 6, 3, 3), (4, 333, "bitpack64", 10, 10, 5), (12, 400, "bitpack64", 5, 2, 1),
        (8, 2050, "int8", 8, 0, 4)]


def run_alone(pam, i, spec):
    L, R, layout, nt, ns, _ = spec
    J = pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(6, i))
    p = pam.Population(L, R, J, pa_inputs.population_seed(6, i, 0), layout=layout)
    obs = []
    for b in linear(5.0, nt)[1:]:
        p.resample(b)
        p.sweep(b, ns)
        obs.append(p.observables())
    st = p.export_state()
    p.close()
    return obs, st


def test_stepper_matches_single_calls(pam):
    import torch

    stream = torch.cuda.Stream()
    stepper = pam.Stepper(8, 12, stream)
    active = []    # [index, population, schedule, k]
    out = {i: [] for i in range(len(SPEC))}
    states = {}
    tick = 0
    while tick < 3 or active:
        for i, s in enumerate(SPEC):
            if s[5] == tick:
                L, R, layout = s[0], s[1], s[2]
                J = pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(6, i))
                pop = pam.Population(L, R, J, pa_inputs.population_seed(6, i, 0), layout=layout,
                                     stream=stream)
                active.append([i, pop, linear(5.0, s[3]), 0])
        if active:
            obs, st = stepper.step([a[1] for a in active], [a[2][a[3] + 1] for a in active],
                                   [SPEC[a[0]][4] for a in active])
            assert np.all(st == 0)
            still = []
            for a, o in zip(active, obs):
                out[a[0]].append(o)
                a[3] += 1
                if a[3] == len(a[2]) - 1:
                    # the instance is its own again: its own observables agree
                    o2 = a[1].observables()
                    for f in FIELDS:
                        assert o2[f] == o[f], (a[0], f)
                    states[a[0]] = a[1].export_state()
                    a[1].close()
                else:
                    still.append(a)
            active = still
        tick += 1
    stepper.close()
    for i, s in enumerate(SPEC):
        ref, st = run_alone(pam, i, s)
        assert len(out[i]) == len(ref) == s[3] - 1
        for k, (a, b) in enumerate(zip(ref, out[i])):
            for f in FIELDS:
                assert a[f] == b[f], (i, k, f, a[f], b[f])
        for x, y in zip(st, states[i]):
            np.testing.assert_array_equal(x, y)


def test_stepper_capacity_overflow(pam):
    import torch

    L, R = 4, 256
    J = pa_inputs.couplings_pm(L, 8)
    betas = list(np.linspace(0.0, 5.0, 41))
    stream = torch.cuda.Stream()
    stepper = pam.Stepper(4, 8, stream)
    tight = pam.Population(L, R, J, 5, capacity=R, layout="int8", stream=stream)
    roomy = pam.Population(L, R, J, 6, layout="int8", stream=stream)
    ref = pam.Population(L, R, J, 5, capacity=R, layout="int8")
    failed_at = None
    for k in range(1, len(betas)):
        pops = [roomy] if failed_at else [tight, roomy]
        obs, st = stepper.step(pops, [betas[k]] * len(pops), [1] * len(pops))
        assert st[-1] == 0
        if failed_at is None:
            try:
                ref.resample(betas[k])
                ref.sweep(betas[k], 1)
                assert st[0] == 0
                assert ref.observables()["beta_F"] == obs[0]["beta_F"]
            except pam.PAError as e:
                assert e.status == pam.PA_ECAPACITY and st[0] == pam.PA_ECAPACITY
                failed_at = k
    assert failed_at is not None and failed_at > 1
    for x, y in zip(ref.export_state(), tight.export_state()):
        np.testing.assert_array_equal(x, y)
    # the failed instance can go on by itself (same state, same counters)
    tight.sweep(betas[failed_at - 1], 1)
    ref.sweep(betas[failed_at - 1], 1)
    for x, y in zip(ref.export_state(), tight.export_state()):
        np.testing.assert_array_equal(x, y)
    stepper.close()
    for x in (tight, roomy, ref):
        x.close()


def test_stepper_errors(pam):
    import torch

    stream = torch.cuda.Stream()
    J = pa_inputs.couplings_pm(4, 1)
    with pytest.raises(pam.PAError):
        pam.Stepper(0, 8, stream)
    st = pam.Stepper(2, 6, stream)
    other = pam.Population(4, 200, J, 1)                  # default stream
    big = pam.Population(8, 200, pa_inputs.couplings_pm(8, 1), 2, stream=stream)
    a = pam.Population(4, 200, J, 3, stream=stream)
    for pops in ([other], [big], [a, a]):
        with pytest.raises(pam.PAError) as e:
            st.step(pops, [0.1] * len(pops), [1] * len(pops))
        assert e.value.status == pam.PA_EINVAL
    with pytest.raises(pam.PAError) as e:
        st.step([a, a, a], [0.1] * 3, [1] * 3)                # more than max_pops
    assert e.value.status == pam.PA_EINVAL
    a.resample(0.1)                                           # pending copy step
    with pytest.raises(pam.PAError) as e:
        st.step([a], [0.2], [1])
    assert e.value.status == pam.PA_ESTATE
    st.close()
    for x in (other, big, a):
        x.close()


def make_requests(spec):
    from paper_1711_02146_amd.serve import Request

    out = []
    for i, (arrival, L, R, nt) in enumerate(spec):
        out.append(Request(rid=i, arrival=arrival, L=L, R=R, n_temps=nt, n_sweeps=10, beta_max=5.0,
                           J=pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(7, i)),
                           seed=pa_inputs.population_seed(7, i, 0)))
    return out


def test_served_results_same_alone_and_in_mix(pam):
    from paper_1711_02146_amd.serve import Server

    spec = [(0.0, 4, 3000, 21), (0.02, 6, 1200, 11), (0.03, 8, 900, 16), (0.05, 10, 500, 9),
            (0.05, 12, 300, 7), (0.15, 4, 5000, 13)]
    reqs = make_requests(spec)
    srv = Server(hbm_budget=8 << 30, max_active=8, max_L=12, keep_trajectory=True)
    mixed = srv.run(reqs, realtime=False, tick_dt=0.01)
    assert max(srv.tick_sizes) >= 4      # several requests shared launches
    srv.close()
    for r, m in zip(reqs, mixed):
        assert m.status == 0 and len(m.trajectory) == r.n_temps - 1
        alone_srv = Server(hbm_budget=8 << 30, max_active=1, max_L=12, keep_trajectory=True)
        (a,) = alone_srv.run([r], realtime=False, tick_dt=0.01)
        alone_srv.close()
        assert a.status == 0
        for k, (x, y) in enumerate(zip(a.trajectory, m.trajectory)):
            for f in FIELDS:
                assert x[f] == y[f], (r.rid, k, f)
        assert a.attempts == m.attempts
