"""The C ABI library loads and exports every entry point include/pa.h declares
(host-only checks; no GPU work is issued)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pa.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(pa_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for need in ("pa_init_instance", "pa_sweep", "pa_resample", "pa_observables",
                 "pa_choose_beta", "pa_overlap_hist", "pa_workspace_bytes", "pa_free"):
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_1711_02146_amd as pam

    lib = ctypes.CDLL(pam.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(pam.EXPORTED) == set(declared())


def test_workspace_sizing_and_argument_checks():
    import paper_1711_02146_amd as pam

    p = pam.pa_params(L=10, R=500000, capacity=0, layout=pam.PA_LAYOUT_BITPACK64, seed=1,
                      flags=0, model=0)
    nb = pam.pa_workspace_bytes(p)
    # two bit-packed buffers of ceil(cap/64) tiles x N x 8 bytes dominate
    cap = 500000 + 16 * 707 + 256
    assert nb >= 2 * (cap // 64) * 1000 * 8
    assert nb < 200 * 2 ** 20
    for bad in (dict(L=5), dict(L=2), dict(L=18), dict(R=0), dict(layout=7), dict(flags=8),
                dict(flags=0x80000000), dict(capacity=10), dict(model=3)):
        q = pam.pa_params(L=10, R=1000, capacity=0, layout=1, seed=1, flags=0, model=0)
        for k, v in bad.items():
            setattr(q, k, v)
        assert pam.pa_workspace_bytes(q) == 0, bad
    # Gaussian couplings keep a histogram over every possible E16 window
    g = pam.pa_params(L=10, R=1000, capacity=0, layout=2, seed=1, flags=0, model=1)
    q = pam.pa_params(L=10, R=1000, capacity=0, layout=2, seed=1, flags=0, model=0)
    assert pam.pa_workspace_bytes(g) >= pam.pa_workspace_bytes(q) + 16 * (6 * 1000 * 127 - 3 * 1000)
    # the debugging flags change nothing in the workspace
    for flags in (pam.PA_FLAG_CHECK_ENERGY, pam.PA_FLAG_FAULT_HOOK, pam.PA_FLAG_TIME_SWEEPS,
                  pam.PA_FLAG_CHECK_ENERGY | pam.PA_FLAG_FAULT_HOOK):
        f = pam.pa_params(L=10, R=500000, capacity=0, layout=pam.PA_LAYOUT_BITPACK64, seed=1,
                          flags=flags, model=0)
        assert pam.pa_workspace_bytes(f) == nb
    assert pam.pa_strerror(pam.PA_ECAPACITY) == "resampled population exceeds capacity"
    assert pam.pa_strerror(pam.PA_ECHECK).startswith("energy check failed")
    assert pam.lib().pa_debug_inject(None, pam.PA_INJECT_FAIL_AFTER, 1) == pam.PA_EINVAL
    with pytest.raises(pam.PAError):
        pam.pa_init_instance(p, np.ones(3000, np.int8), 0, 0, 0)  # null workspace: PA_EINVAL


def test_make_couplings_pm_host_call():
    """The library's host coupling generator (no GPU work) against the
    oracle's, written separately from the same rule; the couplings are +-1
    with probability 1/2 (Sec. II.A)."""
    import oracle
    import paper_1711_02146_amd as pam

    for L, seed in ((2, 0), (3, 1), (4, 0xC0DE0000), (10, 2 ** 63 + 5), (16, 77)):
        J = pam.pa_make_couplings_pm(L, seed)
        np.testing.assert_array_equal(J, oracle.make_couplings_pm(L, seed))
        assert set(np.unique(J)) <= {-1, 1}
    J = pam.pa_make_couplings_pm(16, 12345).astype(np.float64)
    assert abs(J.mean()) < 4.0 / np.sqrt(J.size)
    assert not np.array_equal(pam.pa_make_couplings_pm(8, 1), pam.pa_make_couplings_pm(8, 2))
    assert pam.lib().pa_make_couplings_pm(1, 1, None) == pam.PA_EINVAL
    with pytest.raises(pam.PAError):
        pam.pa_make_couplings_pm(1, 3)


def test_autotune_set_checks_its_arguments():
    """Pinning a sweep form is host bookkeeping (no GPU work)."""
    import paper_1711_02146_amd as pam

    lib = pam.lib()
    assert lib.pa_autotune_set(0, 2, 10, 7813, 8) == pam.PA_OK
    for bad in ((3, 2, 10, 7813, 8), (0, 0, 10, 7813, 8), (0, 2, 5, 7813, 8), (0, 2, 18, 7813, 8),
                (0, 2, 10, 0, 8), (0, 2, 10, 7813, 6)):
        assert lib.pa_autotune_set(*bad) == pam.PA_EINVAL, bad
    assert lib.pa_autotune_reset() == pam.PA_OK


def test_layout_choice_follows_the_layout_table():
    """PA_LAYOUT_AUTO resolves through the autotuner's layout table, keyed by
    (model, L, floor(log2(ceil(R / 64)))), with bit-packing as the built-in
    choice; pinning, lookup and workspace sizing are host bookkeeping."""
    import paper_1711_02146_amd as pam

    lib = pam.lib()
    assert lib.pa_autotune_reset() == pam.PA_OK
    try:
        for L in (4, 6, 8, 10, 12, 16):
            assert pam.pa_layout_choice(L, 100000) == "bitpack64"
            assert pam.pa_layout_choice(L, 100000, "gauss16") == "bitpack64"
        pam.pa_autotune_set_layout(8, 100000, "int8")  # 1563 tiles: size class 10
        assert pam.pa_layout_choice(8, 100000) == "int8"
        assert pam.pa_layout_choice(8, 65537) == "int8"    # 1025 tiles: class 10
        assert pam.pa_layout_choice(8, 65536) == "int8"  # 1024 tiles: class 10
        assert pam.pa_layout_choice(8, 65472) == "bitpack64"  # 1023 tiles: class 9
        assert pam.pa_layout_choice(8, 131073) == "bitpack64"  # 2049 tiles: class 11
        assert pam.pa_layout_choice(8, 50000) == "bitpack64"  # 782 tiles: class 9
        assert pam.pa_layout_choice(10, 100000) == "bitpack64"
        assert pam.pa_layout_choice(8, 100000, "gauss16") == "bitpack64"

        def ws(layout, R=100000, L=8):
            return pam.pa_workspace_bytes(pam.pa_params(L=L, R=R, capacity=0, layout=layout,
                                                        seed=1, flags=0, model=0))

        assert ws(pam.PA_LAYOUT_AUTO) == ws(pam.PA_LAYOUT_INT8) > ws(pam.PA_LAYOUT_BITPACK64)
        assert ws(pam.PA_LAYOUT_AUTO, R=50000) == ws(pam.PA_LAYOUT_BITPACK64, R=50000)
        p = pam.pa_params(L=8, R=100000, capacity=0, layout=pam.PA_LAYOUT_BITPACK64, seed=1,
                          flags=pam.PA_FLAG_FAULT_HOOK, model=0)
        assert lib.pa_autotune_layout_workspace_bytes(ctypes.byref(p)) == ws(pam.PA_LAYOUT_INT8)
        p.L = 7
        assert lib.pa_autotune_layout_workspace_bytes(ctypes.byref(p)) == 0
        assert lib.pa_autotune_reset() == pam.PA_OK
        assert pam.pa_layout_choice(8, 100000) == "bitpack64"
        out = ctypes.c_uint32(0)
        for bad in ((3, 8, 1000), (0, 7, 1000), (0, 2, 1000), (0, 18, 1000), (0, 8, 0)):
            assert lib.pa_layout_choice(*bad, ctypes.byref(out)) == pam.PA_EINVAL, bad
        assert lib.pa_layout_choice(0, 8, 1000, None) == pam.PA_EINVAL
        for bad in ((3, 8, 16, 1), (0, 8, 16, 0), (0, 8, 16, 3), (0, 9, 16, 1), (0, 8, 0, 1)):
            assert lib.pa_autotune_set_layout(*bad) == pam.PA_EINVAL, bad
        assert lib.pa_autotune_layout(None, None, None, 0, None, 1.0, 10, 3, None,
                                      None) == pam.PA_EINVAL
    finally:
        lib.pa_autotune_reset()


def test_real_coupling_model_sizing_and_argument_checks():
    """PA_MODEL_GAUSS: int64 energy words, the he and threshold tables of every
    (site, pattern) and one reduction partial per slot block; the creation
    call rejects bad couplings before any device work."""
    import paper_1711_02146_amd as pam

    L, R = 10, 100000
    q = pam.pa_params(L=L, R=R, capacity=0, layout=2, seed=1, flags=0, model=0)
    g = pam.pa_params(L=L, R=R, capacity=0, layout=2, seed=1, flags=0, model=pam.PA_MODEL_GAUSS)
    cap = R + 16 * 316 + 256
    cap = (cap + 255) // 256 * 256
    extra = pam.pa_workspace_bytes(g) - pam.pa_workspace_bytes(q)
    # (less the +-J histogram and resampling table of 3N + 1 levels)
    assert extra >= 2 * cap * 4 + 2 * L ** 3 * 64 * 8 + (cap // 256) * 32 - 20 * 3001 - 8192
    lib = pam.lib()
    out = ctypes.c_void_p()
    good = np.ldexp(np.rint(np.ldexp(np.linspace(-3, 3, 3 * L ** 3), 32)), -32)
    for J in (np.where(np.arange(3000) == 7, np.nan, good), np.where(np.arange(3000) == 5, 8.0, good),
              np.where(np.arange(3000) == 5, -np.inf, good)):
        J = np.ascontiguousarray(J, np.float64)
        assert lib.pa_init_instance_real(ctypes.byref(g), J.ctypes.data, 256, 1 << 30, None,
                                         ctypes.byref(out)) == pam.PA_EINVAL
    # the real-coupling model takes FP64 couplings only, and only them
    J8 = np.ones(3 * L ** 3, np.int8)
    assert lib.pa_init_instance(ctypes.byref(g), J8.ctypes.data, 256, 1 << 30, None,
                                ctypes.byref(out)) == pam.PA_EINVAL
    assert lib.pa_init_instance_real(ctypes.byref(q), good.ctypes.data, 256, 1 << 30, None,
                                     ctypes.byref(out)) == pam.PA_EINVAL
    assert lib.pa_export_energies(None, None) == pam.PA_ESTATE
