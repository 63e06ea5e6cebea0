"""GPU: the sweep autotuner times both sweep forms and remembers the faster; it
changes neither the population nor any later result (bit-exact against the
oracle afterwards), in the forms it picks for single instances and batches.
The layout autotuner times both spin layouts on a shape; populations created
with layout "auto" then take the faster, and every result is the same under
either choice (against the oracle, bit for bit).  The ceiling probes report
rates within the chip's limits."""
import numpy as np
import pytest

import oracle
import pa_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pam():
    import torch

    assert torch.cuda.is_available()
    import paper_1711_02146_amd as m

    m.lib()
    yield m
    m.pa_autotune_reset()


@pytest.mark.parametrize("L,R,layout", [(8, 30000, "bitpack64"), (6, 5000, "int8")])
def test_autotune_leaves_results_unchanged(pam, L, R, layout):
    pam.pa_autotune_reset()
    J = pa_inputs.couplings_pm(L, 808)
    g = pam.Population(L, R, J, 4242, layout=layout)
    o = oracle.Population(L, J, R, 4242)
    g.resample(0.3)
    o.resample(0.3)
    g.sweep(0.3, 5)
    o.sweep(0.3, 5)
    before = g.export_state()
    obs_before = g.observables()
    t = g.autotune(beta=0.5, n_sweeps=10, repeats=2)
    assert t["split"] in (4, 8)
    assert t["ms_split4"] > 0 and t["ms_split8"] > 0
    assert t["split"] == (8 if t["ms_split8"] < t["ms_split4"] else 4)
    for x, y in zip(before, g.export_state()):
        np.testing.assert_array_equal(x, y)
    assert g.observables() == obs_before
    # later steps (now in the tuned form) stay bit-exact
    for b in (0.6, 0.9):
        g.resample(b)
        o.resample(b)
        g.sweep(b, 10)
        o.sweep(b, 10)
    s, u, f = g.export_state()
    np.testing.assert_array_equal(s.reshape(-1), o.spins)
    np.testing.assert_array_equal(u.astype(np.int32), o.U)
    np.testing.assert_array_equal(f, o.fam)
    g.close()


def test_autotune_needs_no_pending_copy(pam):
    J = pa_inputs.couplings_pm(4, 1)
    g = pam.Population(4, 500, J, 1)
    g.resample(0.2)
    with pytest.raises(pam.PAError) as e:
        g.autotune()
    assert e.value.status == pam.PA_ESTATE
    g.sweep(0.2, 1)
    for beta, n in ((0.5, 0), (-1.0, 10), (float("nan"), 10)):
        with pytest.raises(pam.PAError) as e:
            pam.pa_autotune_sweep(g.handle, beta, n, 1)
        assert e.value.status == pam.PA_EINVAL
    g.close()


def _run_steps(pam, g, o, betas):
    for b in betas:
        g.resample(b)
        g.sweep(b, 10)
        if o is not None:
            o.resample(b)
            o.sweep(b, 10)


def test_autotune_layout_records_a_choice_auto_uses(pam):
    L, R = 6, 6000
    J = pa_inputs.couplings_pm(L, 909)
    pam.pa_autotune_reset()
    try:
        t = pam.pa_autotune_layout(L, R, J, seed=5, beta=0.5, n_sweeps=10, repeats=2)
        assert t["ms_int8"] > 0 and t["ms_bitpack64"] > 0
        assert t["layout"] == ("bitpack64" if t["ms_bitpack64"] <= t["ms_int8"] else "int8")
        assert pam.pa_layout_choice(L, R) == t["layout"]
        g = pam.Population(L, R, J, 77)
        assert g.layout == t["layout"]
        o = oracle.Population(L, J, R, 77)
        _run_steps(pam, g, o, (0.3, 0.7))
        s, u, f = g.export_state()
        np.testing.assert_array_equal(s.reshape(-1), o.spins)
        np.testing.assert_array_equal(u.astype(np.int32), o.U)
        np.testing.assert_array_equal(f, o.fam)
        g.close()
    finally:
        pam.pa_autotune_reset()


@pytest.mark.parametrize("pinned", ["int8", "bitpack64"])
def test_auto_layout_results_identical_under_either_choice(pam, pinned):
    """Pin each layout for one shape: a population created with "auto" takes it,
    and its observables, spins, energies and families after a few steps equal
    those of populations created with either explicit layout."""
    L, R = 8, 9000
    J = pa_inputs.couplings_pm(L, 910)
    pam.pa_autotune_reset()
    try:
        pam.pa_autotune_set_layout(L, R, pinned)
        pops = {"auto": pam.Population(L, R, J, 31)}
        assert pops["auto"].layout == pinned
        for lay in ("int8", "bitpack64"):
            pops[lay] = pam.Population(L, R, J, 31, layout=lay)
        for g in pops.values():
            _run_steps(pam, g, None, (0.4, 0.8, 1.2))
        ref = pops["int8"]
        ref_state = ref.export_state()
        for name, g in pops.items():
            assert g.observables() == ref.observables(), name
            for x, y in zip(ref_state, g.export_state()):
                np.testing.assert_array_equal(x, y, err_msg=name)
        for g in pops.values():
            g.close()
    finally:
        pam.pa_autotune_reset()


def test_autotune_layout_checks_its_workspace(pam):
    import ctypes

    import torch

    L, R = 6, 1000
    J = np.ascontiguousarray(pa_inputs.couplings_pm(L, 1), np.int8)
    p = pam.pa_params(L=L, R=R, capacity=0, layout=0, seed=1, flags=0, model=0)
    need = pam.lib().pa_autotune_layout_workspace_bytes(ctypes.byref(p))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    lib = pam.lib()
    assert lib.pa_autotune_layout(ctypes.byref(p), J.ctypes.data, ws.data_ptr(), need - 256, s,
                                  1.0, 10, 1, None, None) == pam.PA_ENOMEM
    assert lib.pa_autotune_layout(ctypes.byref(p), J.ctypes.data, ws.data_ptr(), need, s,
                                  -1.0, 10, 1, None, None) == pam.PA_EINVAL
    assert lib.pa_autotune_layout(ctypes.byref(p), J.ctypes.data, ws.data_ptr(), need, s,
                                  1.0, 0, 1, None, None) == pam.PA_EINVAL
    pam.pa_autotune_reset()


def test_probe_ceilings(pam):
    """The device ceilings the sweep is measured against.  With one wave
    instruction per SIMD every four cycles, the chip issues 256 CUs x 64 lanes
    x 2.4 GHz = 39.3e12 lane-operations per second; three-source operations
    (v_bfe_u32) stay within that, two-source ones (v_add_u32) may exceed it but
    not the 32 lanes per SIMD per cycle of the packed FP32 peak.  Philox draws
    alone take about ten lane-operations each."""
    c = pam.pa_probe_ceilings()
    peak = 256 * 64 * 2.4e9
    assert 0.5 * peak < c["valu3_lane_ops_per_s"] <= 1.02 * peak
    assert c["valu3_lane_ops_per_s"] <= c["valu_lane_ops_per_s"] <= 2.02 * peak
    assert 1e11 < c["philox_draws_per_s"] < c["valu_lane_ops_per_s"] / 6
    # a missing scratch buffer is refused before any launch
    assert pam.lib().pa_probe_ceilings(None, 0, None, None) == pam.PA_EINVAL
