"""The property helpers used on exported GPU states (tests/props.py) against
the oracle, on random states the test draws itself (CPU)."""
import numpy as np
import pytest

import oracle
import pa_inputs
import props


@pytest.mark.parametrize("L", [3, 4, 6])
def test_props_agree_with_the_oracle(oracle_lib, L):
    N = L ** 3
    rng = np.random.default_rng(40 + L)
    s = rng.choice(np.array([-1, 1], np.int8), (50, N))
    t = rng.choice(np.array([-1, 1], np.int8), (40, N))
    J = pa_inputs.couplings_pm(L, 9)
    np.testing.assert_array_equal(props.unsatisfied_bonds(L, J, s), oracle.energy(L, J, s.reshape(-1)))
    K = pa_inputs.couplings_gauss16(L, 9)
    np.testing.assert_array_equal(props.energy16(L, K, s), oracle.g_energy(L, K, s.reshape(-1)))
    h, _ = oracle.overlap_hist(N, s.reshape(-1), t.reshape(-1))
    np.testing.assert_array_equal(props.overlap_hist65(N, s, t), h)
