"""The C ABI's debugging flags, fault injection and checkpoint/resume.

* PA_FLAG_CHECK_ENERGY recomputes every replica's energy word from its spins
  (the Sec. II.A Hamiltonian) and compares it with the stored word; a run with
  the check on gives the same bits as one without it, and a stored word made
  wrong from the host is reported as PA_ECHECK.
* PA_FLAG_FAULT_HOOK lets pa_debug_inject make a later call fail as a HIP
  error would; everything happens on the host, no kernel is made to fail.
* A population exported after step k (spins, family labels, size, sweep
  counter, step index, beta and the accumulated sum of ln Q of Eq. 9) and
  imported into a fresh instance continues bit for bit as the uninterrupted
  run (Sec. II loop state).
"""
import sys

import numpy as np
import pytest

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
    return m


def _anneal(p, n, eps=0.1, beta_max=5.0, n_sweeps=4):
    out = []
    for _ in range(n):
        b = p.choose_beta(eps, beta_max)
        p.resample(b)
        p.sweep(b, n_sweeps)
        out.append(p.observables())
    return out


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("model", ["pm", "gauss16"])
def test_energy_check_changes_no_bit(pam, layout, model):
    say("energy check", layout, model)
    L, R, seed = 6, 3000, 0x5EED1201
    J = (pa_inputs.couplings_pm(L, 3) if model == "pm" else pa_inputs.couplings_gauss16(L, 3))
    a = pam.Population(L, R, J, seed, layout=layout, model=model)
    b = pam.Population(L, R, J, seed, layout=layout, model=model, flags=pam.PA_FLAG_CHECK_ENERGY)
    ra, rb = _anneal(a, 6), _anneal(b, 6)
    assert ra == rb
    sa, ua, fa = a.export_state()
    sb, ub, fb = b.export_state()
    np.testing.assert_array_equal(sa, sb)
    np.testing.assert_array_equal(ua, ub)
    np.testing.assert_array_equal(fa, fb)
    a.close()
    b.close()


@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
def test_energy_check_finds_a_wrong_word(pam, layout):
    say("energy check finds", layout)
    L, R = 4, 500
    J = pa_inputs.couplings_pm(L, 5)
    flags = pam.PA_FLAG_CHECK_ENERGY | pam.PA_FLAG_FAULT_HOOK
    p = pam.Population(L, R, J, 77, layout=layout, flags=flags)
    _anneal(p, 2)
    pam.pa_debug_inject(p.handle, pam.PA_INJECT_ENERGY, 123)
    with pytest.raises(pam.PAError) as e:
        p.observables()
    assert e.value.status == pam.PA_ECHECK
    with pytest.raises(pam.PAError) as e:
        p.sweep(0.5, 1)
    assert e.value.status == pam.PA_ESTATE  # the instance is unusable from now on
    p.close()
    # without the check the same corruption goes unnoticed (the flag is what finds it)
    q = pam.Population(L, R, J, 77, layout=layout, flags=pam.PA_FLAG_FAULT_HOOK)
    _anneal(q, 2)
    pam.pa_debug_inject(q.handle, pam.PA_INJECT_ENERGY, 123)
    q.observables()
    q.close()


def test_fault_injection_after_n_calls(pam):
    say("fault injection")
    L, R = 4, 400
    J = pa_inputs.couplings_pm(L, 6)
    p = pam.Population(L, R, J, 5, flags=pam.PA_FLAG_FAULT_HOOK)
    other = pam.Population(L, R, J, 6)
    with pytest.raises(pam.PAError) as e:
        pam.pa_debug_inject(other.handle, pam.PA_INJECT_FAIL_AFTER, 0)
    assert e.value.status == pam.PA_EINVAL  # the hook must be enabled at creation
    with pytest.raises(pam.PAError):
        pam.pa_debug_inject(p.handle, 99, 0)
    pam.pa_debug_inject(p.handle, pam.PA_INJECT_FAIL_AFTER, 3)
    b = p.choose_beta(0.1, 5.0)   # 1
    p.resample(b)                 # 2
    p.sweep(b, 2)                 # 3
    with pytest.raises(pam.PAError) as e:
        p.observables()           # 4: fails
    assert e.value.status == pam.PA_EDEVICE
    for call in (lambda: p.observables(), lambda: p.sweep(b, 1), lambda: p.export_state()):
        with pytest.raises(pam.PAError) as e:
            call()
        assert e.value.status == pam.PA_ESTATE
    # another instance on the same device is untouched
    _anneal(other, 2)
    p.close()
    other.close()


def test_fault_injection_in_a_stepper_set(pam):
    import torch

    say("fault injection, stepper")
    L, R = 4, 400
    J = pa_inputs.couplings_pm(L, 8)
    st = torch.cuda.Stream()
    a = pam.Population(L, R, J, 11, stream=st, flags=pam.PA_FLAG_FAULT_HOOK)
    b = pam.Population(L, R, J, 12, stream=st)
    s = pam.Stepper(4, L, st)
    pam.pa_debug_inject(a.handle, pam.PA_INJECT_FAIL_AFTER, 1)
    s.step([a, b], [0.1, 0.1], [2, 2])
    with pytest.raises(pam.PAError) as e:
        s.step([a, b], [0.2, 0.2], [2, 2])
    assert e.value.status == pam.PA_EDEVICE
    # nothing was queued: b continues as if the failed call had not happened
    obs, status = s.step([b], [0.2], [2])
    ref = pam.Population(L, R, J, 12, stream=st)
    s.step([ref], [0.1], [2])
    obs_ref, _ = s.step([ref], [0.2], [2])
    assert obs == obs_ref
    s.close()
    for p in (a, b, ref):
        p.close()


@pytest.mark.parametrize("layout,model", [("bitpack64", "pm"), ("int8", "pm"),
                                          ("bitpack64", "gauss16")])
def test_checkpoint_resume_is_bit_identical(pam, layout, model):
    """Export after step k, import into a fresh instance, finish: every later
    step's scalars and the final population equal the uninterrupted run's."""
    say("checkpoint resume", layout, model)
    L, R, seed, k, n = 8, 6000, 0x5EED1301, 7, 14
    J = (pa_inputs.couplings_pm(L, 9) if model == "pm" else pa_inputs.couplings_gauss16(L, 9))
    full = pam.Population(L, R, J, seed, layout=layout, model=model)
    ref = _anneal(full, n)
    first = pam.Population(L, R, J, seed, layout=layout, model=model)
    head = _anneal(first, k)
    assert head == ref[:k]
    spins, _, fam = first.export_state()
    o = first.observables()
    first.close()
    resumed = pam.Population(L, R, J, seed, layout=layout, model=model)
    resumed.import_state(spins, fam, o["sweeps_done"], o["step"], o["beta"], o["sum_lnQ"])
    tail = _anneal(resumed, n - k)
    for want, got in zip(ref[k:], tail):
        assert got == want
    s1, u1, f1 = full.export_state()
    s2, u2, f2 = resumed.export_state()
    np.testing.assert_array_equal(s1, s2)
    np.testing.assert_array_equal(u1, u2)
    np.testing.assert_array_equal(f1, f2)
    full.close()
    resumed.close()


# ---------------------------------------------------------------------------
# pa_anneal_step: one whole step with a single synchronisation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("model", ["pm", "gauss16"])
def test_anneal_step_equals_separate_calls(pam, layout, model):
    say("anneal step", layout, model)
    L, R, seed = 8, 9000, 0x5EED1401
    J = (pa_inputs.couplings_pm(L, 4) if model == "pm" else pa_inputs.couplings_gauss16(L, 4))
    a = pam.Population(L, R, J, seed, layout=layout, model=model)
    b = pam.Population(L, R, J, seed, layout=layout, model=model,
                       flags=pam.PA_FLAG_TIME_SWEEPS)
    ref = _anneal(a, 8)
    for k in range(8):
        beta, obs = b.anneal_step(0.1, 5.0, 4)
        assert beta == ref[k]["beta"], k
        assert obs["sweep_ms"] > 0.0
        obs["sweep_ms"] = 0.0
        assert obs == ref[k], k
    # fixed temperatures (eps_target < 0): the step to the given beta
    for beta in (0.9, 1.3):
        a.resample(beta)
        a.sweep(beta, 3)
        want = a.observables()
        got = b.step_to(beta, 3)
        got["sweep_ms"] = 0.0
        assert got == want
    s1, u1, f1 = a.export_state()
    s2, u2, f2 = b.export_state()
    np.testing.assert_array_equal(s1, s2)
    np.testing.assert_array_equal(u1, u2)
    np.testing.assert_array_equal(f1, f2)
    a.close()
    b.close()


def test_anneal_step_against_oracle(pam):
    import oracle

    say("anneal step vs oracle")
    L, R, seed = 6, 4000, 0x5EED1501
    J = pa_inputs.couplings_pm(L, 21)
    g = pam.Population(L, R, J, seed, layout="bitpack64")
    o = oracle.Population(L, J, R, seed)
    for k in range(12):
        beta, obs = g.anneal_step(0.1, 5.0, 5)
        bo = o.choose_beta(0.1, 5.0)
        assert beta == bo, k
        o.resample(bo)
        o.sweep(bo, 5)
        rec = o.observables()
        for key in ("beta_F", "mean_E", "rho_t", "lnQ", "eps_expected"):
            assert obs[key] == getattr(rec, key), (k, key)
        assert obs["R_tilde"] == rec.R_tilde and obs["sum_eta2"] == rec.sum_eta2
    s, u, f = g.export_state()
    np.testing.assert_array_equal(s.reshape(-1), o.spins)
    np.testing.assert_array_equal(u.astype(np.int32), o.U)
    np.testing.assert_array_equal(f, o.fam)
    g.close()


@pytest.mark.parametrize("model", ["pm", "gauss16"])
def test_anneal_step_overflow_keeps_population(pam, model):
    """With capacity R, a large step overflows: PA_ECAPACITY, and the
    population, its counters and its next steps are as if it had not been tried."""
    say("anneal step overflow", model)
    L, R = 4, 256
    J = (pa_inputs.couplings_pm(L, 8) if model == "pm" else pa_inputs.couplings_gauss16(L, 8))
    g = pam.Population(L, R, J, 5, capacity=R, layout="int8", model=model)
    failed = False
    for beta in np.linspace(0.5, 5.0, 40):
        before, obs_before = g.export_state(), g.observables()
        try:
            g.step_to(float(beta), 1)
        except pam.PAError as e:
            assert e.status == pam.PA_ECAPACITY
            failed = True
            break
    assert failed
    for x, y in zip(before, g.export_state()):
        np.testing.assert_array_equal(x, y)
    assert g.observables() == obs_before
    g.close()


# ---------------------------------------------------------------------------
# pa_anneal_run: many steps per call, pipelined
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("layout", ["int8", "bitpack64"])
@pytest.mark.parametrize("model", ["pm", "gauss16"])
def test_anneal_run_equals_separate_calls_to_the_end(pam, layout, model):
    """A whole anneal to beta = 5 in chunks of steps: every step's scalars,
    and the final population, equal the separate calls'."""
    say("anneal run", layout, model)
    L, R, seed = 6, 3000, 0x5EED1601
    J = (pa_inputs.couplings_pm(L, 14) if model == "pm" else pa_inputs.couplings_gauss16(L, 14))
    a = pam.Population(L, R, J, seed, layout=layout, model=model)
    b = pam.Population(L, R, J, seed, layout=layout, model=model, flags=pam.PA_FLAG_TIME_SWEEPS)
    ref = []
    while not ref or ref[-1]["beta"] < 5.0:
        ref += _anneal(a, 1, n_sweeps=3)
    got = []
    while not got or got[-1]["beta"] < 5.0:
        chunk = b.anneal_run(0.1, 5.0, 3, 17)
        assert 1 <= len(chunk) <= 17
        got += chunk
    assert len(got) == len(ref)
    for k, (x, y) in enumerate(zip(got, ref)):
        assert x["sweep_ms"] > 0.0
        x["sweep_ms"] = 0.0
        assert x == y, k
    with pytest.raises(pam.PAError) as e:
        b.anneal_run(0.1, 5.0, 3, 4)  # beta_max reached: no step left
    assert e.value.status == pam.PA_EINVAL
    for x, y in zip(a.export_state(), b.export_state()):
        np.testing.assert_array_equal(x, y)
    a.close()
    b.close()


def test_anneal_run_stops_at_an_overflow(pam):
    """With capacity R some step overflows: the steps before it stand (equal
    to the separate calls), the call reports PA_ECAPACITY, and the population
    is as after the last step taken."""
    say("anneal run overflow")
    L, R = 4, 256
    J = pa_inputs.couplings_pm(L, 18)
    a = pam.Population(L, R, J, 9, capacity=R, layout="int8")
    b = pam.Population(L, R, J, 9, capacity=R, layout="int8")
    with pytest.raises(pam.PAError) as e:
        b.anneal_run(0.3, 5.0, 2, 400)
    assert e.value.status == pam.PA_ECAPACITY
    taken = e.value.steps
    ref = _anneal(a, len(taken), eps=0.3, n_sweeps=2)
    assert taken == ref
    with pytest.raises(pam.PAError) as e2:
        _anneal(a, 1, eps=0.3, n_sweeps=2)
    assert e2.value.status == pam.PA_ECAPACITY
    for x, y in zip(a.export_state(), b.export_state()):
        np.testing.assert_array_equal(x, y)
    assert a.observables() == b.observables()
    a.close()
    b.close()
