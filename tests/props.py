"""Properties that hold at any population size, checked on states the GPU
exported after a whole anneal (where the oracle cannot replay the history):
plain numpy restatements of the energy and overlap definitions of Sec. II.A
(Amey & Machta, arXiv:1711.02146), written here so that no value the GPU
produced is ever fed to the oracle.

Layout: spins [replica][site] int8 +-1, site = x + L (y + L z); coupling
J[d N + site] joins site and site + e_d (d = 0, 1, 2 for x, y, z)."""
import numpy as np


def _bond_products(L: int, spins: np.ndarray):
    """s_site * s_(site + e_d) for d = 0, 1, 2: three arrays [R][N]."""
    s = np.asarray(spins, np.int32).reshape(-1, L, L, L)  # [r][z][y][x]
    out = []
    for axis in (3, 2, 1):  # x, y, z
        out.append((s * np.roll(s, -1, axis=axis)).reshape(s.shape[0], -1))
    return out


def unsatisfied_bonds(L: int, J: np.ndarray, spins: np.ndarray) -> np.ndarray:
    """+-J: the number of bonds with J s s = -1, per replica."""
    N = L ** 3
    J = np.asarray(J, np.int32)
    prods = _bond_products(L, spins)
    return sum((J[d * N:(d + 1) * N][None, :] * prods[d] < 0).sum(axis=1)
               for d in range(3)).astype(np.int32)


def energy16(L: int, K: np.ndarray, spins: np.ndarray) -> np.ndarray:
    """Couplings k = 16 J: E16 = -sum_b k_b s s, per replica."""
    N = L ** 3
    K = np.asarray(K, np.int64)
    prods = _bond_products(L, spins)
    return (-sum((K[d * N:(d + 1) * N][None, :] * prods[d]).sum(axis=1)
                 for d in range(3))).astype(np.int32)


def overlap_hist65(N: int, sa: np.ndarray, sb: np.ndarray) -> np.ndarray:
    """65-bin spin-overlap histogram of replica i of a against replica i of b:
    d differing sites, bin = (128 (N - d) + N) // (2N)."""
    n = min(sa.shape[0], sb.shape[0])
    d = (np.asarray(sa[:n]) != np.asarray(sb[:n])).sum(axis=1).astype(np.int64)
    return np.bincount((128 * (N - d) + N) // (2 * N), minlength=65).astype(np.uint64)
