"""pa_link_overlap_hist_noalloc (scratch in a fixed device array of the
library, no allocation) against pa_link_overlap_hist (scratch in the
instance's workspace), through the C ABI: the link-overlap counts of two
populations of one sample (Sec. II.A, q_l = 1 - 2 D / 3N), on two calls in a
row, the second with a smaller input, and the rejection of a lattice larger
than the fixed array holds.
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


def _pair(pam, L, R, layout, model, cseed, seed):
    J = pa_inputs.couplings_pm(L, cseed) if model == "pm" else pa_inputs.couplings_gauss16(L, cseed)
    a = pam.Population(L, R, J, seed, layout=layout, model=model)
    b = pam.Population(L, R + 37, J, seed + 1, layout=layout, model=model)
    for p in (a, b):
        p.step_to(0.4, 3)
    return a, b


def test_noalloc_link_overlap_equals_workspace_version(pam):
    lib = pam.lib()
    # first call: L = 12, the largest lattice the array holds (5185 bins)
    say("no-alloc link overlap, L=12")
    a, b = _pair(pam, 12, 9000, "bitpack64", "pm", 31, 0x5EED1701)
    nbins = 3 * 12 ** 3 + 1
    assert nbins == pam.PA_NOALLOC_MAX_BINS
    want = pam.pa_link_overlap_hist(a.handle, b.handle, nbins)
    got = pam.pa_link_overlap_hist_noalloc(a.handle, b.handle, nbins)
    np.testing.assert_array_equal(got, want)
    assert int(got.sum()) == min(a.observables()["R_tilde"], b.observables()["R_tilde"])
    a.close()
    b.close()
    # second call, smaller input: L = 6, int8, Gaussian couplings; the array
    # still holds the first call's counts, which must not leak into these
    say("no-alloc link overlap, L=6")
    a, b = _pair(pam, 6, 1500, "int8", "gauss16", 32, 0x5EED1801)
    nbins = 3 * 6 ** 3 + 1
    want = pam.pa_link_overlap_hist(a.handle, b.handle, nbins)
    got = pam.pa_link_overlap_hist_noalloc(a.handle, b.handle, nbins)
    np.testing.assert_array_equal(got, want)
    # argument checks as the workspace version
    assert lib.pa_link_overlap_hist_noalloc(a.handle, b.handle, nbins + 1,
                                            got.ctypes.data) == pam.PA_EINVAL
    assert lib.pa_link_overlap_hist_noalloc(a.handle, a.handle, nbins,
                                            got.ctypes.data) == pam.PA_EINVAL
    a.close()
    b.close()


def test_noalloc_rejects_lattices_beyond_the_array(pam):
    """L = 14 needs 8233 bins: PA_ENOMEM, decided on the host before any work."""
    say("no-alloc link overlap, L=14 rejected")
    lib = pam.lib()
    J = pa_inputs.couplings_pm(14, 33)
    a = pam.Population(14, 100, J, 1)
    b = pam.Population(14, 100, J, 2)
    h = np.zeros(3 * 14 ** 3 + 1, np.uint64)
    assert lib.pa_link_overlap_hist_noalloc(a.handle, b.handle, h.size,
                                            h.ctypes.data) == pam.PA_ENOMEM
    # the instances stay usable
    want = pam.pa_link_overlap_hist(a.handle, b.handle, h.size)
    assert int(want.sum()) == 100
    a.close()
    b.close()
