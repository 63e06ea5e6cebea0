"""Pins of the oracle's use of its random numbers, against rocRAND's
open-source Philox4x32-10 engine run on the host (tests/philox_rocrand_ref.cpp).

Every draw of the method is one word of Philox4x32-10 (Salmon et al., SC'11)
under the population seed (or the coupling seed), at a counter whose layout
the library and the oracle share as a contract.  test_oracle_pins checks the
oracle's generator itself; here each place the oracle draws from it is
recomputed from rocRAND's outputs and a restatement of the rule, written in
this file:

  couplings (Sec. II.A, +-J with p = 1/2): J_b = -1 iff bit 31 of word b & 3
      of Philox(coupling_seed; b >> 2, 0, 0, TAG_J);
  initial spins (Sec. II, beta = 0): s = -1 iff bit 31 of word site & 3 of
      Philox(seed; r, site >> 2, 0, TAG_INIT);
  copy counts (Sec. II, nearest-integer resampling): u53 = (w0 << 21) |
      (w1 >> 11) of Philox(seed; i, k, 0, TAG_RES), n_i = fl + [u53 < T];
  Metropolis (Sec. II MCMC): for colour 0 then 1, a move raising the energy
      by dE is taken iff word cm & 3 of Philox(seed; slot, t, cm >> 2, TAG_MET)
      is below floor(2^32 exp(-beta dE)), cm = c N / 2 + (site >> 1).

The Metropolis pin is a brute-force sweep of a few L = 4 replicas in plain
Python.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import pa_inputs

HERE = os.path.dirname(os.path.abspath(__file__))
TAG_J, TAG_INIT, TAG_MET, TAG_RES = 0x434F5550, 0x494E4954, 0x4D455452, 0x52455341


@pytest.fixture(scope="module")
def rocrand(tmp_path_factory, oracle_lib):
    gxx = shutil.which("g++")
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    assert gxx and os.path.exists(hdr), "g++ and rocRAND headers are needed for these pins"
    exe = tmp_path_factory.mktemp("rocrand") / "philox_ref"
    subprocess.check_call([gxx, "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           os.path.join(HERE, "philox_rocrand_ref.cpp"), "-o", str(exe)])

    def run(counters, seed):
        """Philox4x32-10 words of each counter (c0, c1, c2, c3) under the 64-bit key."""
        k0, k1 = seed & 0xFFFFFFFF, seed >> 32
        text = "".join("%x %x %x %x %x %x\n" % (*c, k0, k1) for c in counters)
        out = subprocess.run([str(exe)], input=text, capture_output=True, text=True,
                             check=True).stdout
        words = [[int(w, 16) for w in line.split()] for line in out.strip().splitlines()]
        assert len(words) == len(counters)
        return np.array(words, dtype=np.uint64)

    return run


# A population seed whose Metropolis stream holds the draw 2^32 - 1 in its
# first sweep: replica 58, site group 0, word 0 (the site at colour-major
# index 0).  The real-coupling GPU test of that draw relies on it.
SEED_TOP_DRAW = 0x5EED0000000C56F4


def test_top_draw_seed(rocrand):
    w = rocrand([(58, 0, 0, TAG_MET)], SEED_TOP_DRAW)
    assert int(w[0][0]) == 0xFFFFFFFF


@pytest.mark.parametrize("L,seed", [(3, 1), (4, 0xC0DE0000), (10, 2 ** 63 + 5)])
def test_couplings_counter_layout(rocrand, L, seed):
    nb = 3 * L ** 3
    w = rocrand([(g, 0, 0, TAG_J) for g in range((nb + 3) // 4)], seed)
    bits = (w.reshape(-1)[:nb] >> 31) & 1
    want = np.where(bits == 1, -1, 1).astype(np.int8)
    np.testing.assert_array_equal(oracle.make_couplings_pm(L, seed), want)


def test_init_counter_layout(rocrand):
    L, R, seed = 4, 5, 0x5EED0042
    N = L ** 3
    o = oracle.Population(L, pa_inputs.couplings_pm(L, 7), R, seed)
    w = rocrand([(r, g, 0, TAG_INIT) for r in range(R) for g in range(N // 4)], seed)
    bits = ((w.reshape(R, N) >> 31) & 1).astype(np.int64)
    np.testing.assert_array_equal(o.spins.reshape(R, N), np.where(bits == 1, -1, 1))


def test_copy_count_counter_layout(rocrand):
    """The copy rule with rocRAND's words, for a table whose fractional parts
    make the extra copy a coin flip at every level."""
    seed, step = 0x5EED0777, 3
    rng = np.random.default_rng(5)
    n_levels = 40
    U = rng.integers(0, n_levels, 400).astype(np.int32)
    fl = rng.integers(0, 3, n_levels).astype(np.uint32)
    T = rng.integers(0, 2 ** 53, n_levels, dtype=np.uint64)
    w = rocrand([(i, step, 0, TAG_RES) for i in range(U.size)], seed)
    u53 = (w[:, 0] << np.uint64(21)) | (w[:, 1] >> np.uint64(11))
    want = fl[U] + (u53 < T[U]).astype(np.uint32)
    np.testing.assert_array_equal(oracle.copy_counts(U, fl, T, seed, step), want)


def _brute_force_sweeps(L, J, spins, seed, beta, t0, n_sweeps, draws):
    """Checkerboard Metropolis, one site and replica at a time, in plain Python."""
    N = L ** 3
    s = spins.astype(np.int64).copy()
    R = s.shape[0]
    thr = {dE: math.floor(math.ldexp(math.exp(-beta * dE), 32)) for dE in (4, 8, 12)}

    def site(x, y, z):
        return (x % L) + L * ((y % L) + L * (z % L))

    for t in range(t0, t0 + n_sweeps):
        for colour in (0, 1):
            for z in range(L):
                for y in range(L):
                    for x in range(L):
                        if (x + y + z) % 2 != colour:
                            continue
                        i = site(x, y, z)
                        # bond d*N + site joins site and site + e_d
                        bonds = [(J[0 * N + i], site(x + 1, y, z)), (J[0 * N + site(x - 1, y, z)], site(x - 1, y, z)),
                                 (J[1 * N + i], site(x, y + 1, z)), (J[1 * N + site(x, y - 1, z)], site(x, y - 1, z)),
                                 (J[2 * N + i], site(x, y, z + 1)), (J[2 * N + site(x, y, z - 1)], site(x, y, z - 1))]
                        cm = colour * (N // 2) + (i >> 1)
                        for r in range(R):
                            h = sum(int(j) * int(s[r, n]) for j, n in bonds)
                            dE = 2 * int(s[r, i]) * h
                            if dE > 0 and not int(draws[(r, t, cm >> 2)][cm & 3]) < thr[dE]:
                                continue
                            s[r, i] = -s[r, i]
    return s


@pytest.mark.parametrize("beta", [0.35, 1.2])
def test_metropolis_counter_layout(rocrand, beta):
    L, R, seed, n_sweeps = 4, 3, 0x5EED0901, 2
    N = L ** 3
    J = pa_inputs.couplings_pm(L, 11)
    o = oracle.Population(L, J, R, seed)
    o.sweep(0.1, 1)  # the sweep counter t moves on: the pinned sweeps start at t = 1
    start = o.spins.reshape(R, N).copy()
    keys = [(r, t, g) for r in range(R) for t in range(1, 1 + n_sweeps) for g in range(N // 4)]
    w = rocrand([(r, t, g, TAG_MET) for (r, t, g) in keys], seed)
    draws = {k: w[i] for i, k in enumerate(keys)}
    want = _brute_force_sweeps(L, J, start, seed, beta, 1, n_sweeps, draws)
    o.sweep(beta, n_sweeps)
    np.testing.assert_array_equal(o.spins.reshape(R, N), want)
    # the energy words follow the spins (U = unsatisfied bonds)
    np.testing.assert_array_equal(o.U, oracle.energy(L, J, want.astype(np.int8)))
    assert not np.array_equal(want, start)
