"""Exact thermodynamics of small lattices (test infrastructure).

Two independent exact routes for checking the PA oracle:

* ``density_of_states`` (C, Gray-code enumeration of all 2^N states) gives
  Z(beta) = sum_U g(U) exp(-beta E(U)) with E = 2U - 3N, hence beta F = -ln Z,
  <E> and var(E) at any beta (Sec. II.A model, Sec. II.A free energy).
* ``TransferMatrixL3`` (numpy, FP64) builds the 512x512 layer transfer
  matrices of the L = 3 periodic lattice and returns Z and every pair
  correlation C_nm = <s_n s_m>; from these <q^2> = (1/N^2) sum_nm C_nm^2
  for two independent replicas (Sec. II.A spin overlap), and
  <E> = -sum_bonds J <s_i s_j> as a cross-check of the enumeration.
"""
from __future__ import annotations

import math

import numpy as np

from . import density_of_states


def thermo_from_dos(g: np.ndarray, N: int, beta: float):
    """(ln Z, <E>, var E) at beta from the density of states g[U]."""
    U = np.arange(g.size, dtype=np.float64)
    E = 2.0 * U - 3.0 * N
    mask = g > 0
    logw = np.log(g[mask].astype(np.float64)) - beta * E[mask]
    m = logw.max()
    w = np.exp(logw - m)
    Zs = w.sum()
    lnZ = m + math.log(Zs)
    Em = float((w * E[mask]).sum() / Zs)
    E2 = float((w * E[mask] ** 2).sum() / Zs)
    return lnZ, Em, E2 - Em * Em


class TransferMatrixL3:
    """Exact Z and <s_n s_m> for L = 3 with periodic boundaries."""

    L = 3
    N = 27

    def __init__(self, J: np.ndarray):
        J = np.asarray(J, np.float64)
        assert J.size == 81
        self.J = J
        L, N = 3, 27
        a = np.arange(512)
        # spin of plaquette position p = x + 3y in layer state a: bit set -> -1
        self.S = 1 - 2 * ((a[:, None] >> np.arange(9)[None, :]) & 1)  # (512, 9)
        self.intra = np.zeros((3, 512))
        self.inter = np.zeros((3, 512, 512))
        for z in range(3):
            e = np.zeros(512)
            for y in range(3):
                for x in range(3):
                    p = x + 3 * y
                    site = x + L * (y + L * z)
                    px = ((x + 1) % 3) + 3 * y
                    py = x + 3 * ((y + 1) % 3)
                    e -= J[0 * N + site] * self.S[:, p] * self.S[:, px]
                    e -= J[1 * N + site] * self.S[:, p] * self.S[:, py]
            self.intra[z] = e
            jz = np.array([J[2 * N + (p % 3) + L * ((p // 3) + L * z)] for p in range(9)])
            # V_z(a, b) = -sum_p Jz_p s_p(a) s_p(b), b is layer z+1
            self.inter[z] = -(self.S * jz[None, :]) @ self.S.T

    def _mats(self, beta):
        mats, shifts = [], []
        for z in range(3):
            x = -beta * (self.intra[z][:, None] + self.inter[z])
            c = x.max()
            mats.append(np.exp(x - c))
            shifts.append(c)
        return mats, shifts

    def lnZ(self, beta: float) -> float:
        M, c = self._mats(beta)
        P = M[0] @ M[1] @ M[2]
        return math.log(np.trace(P)) + sum(c)

    def correlations(self, beta: float) -> np.ndarray:
        """C[n, m] = <s_n s_m>, sites numbered x + 3(y + 3z)."""
        M, _ = self._mats(beta)
        N = 27
        C = np.zeros((N, N))

        def prod(z0, z1):  # M_{z0} M_{z0+1} ... M_{z1-1} (cyclic), identity if z0 == z1
            P = np.eye(512)
            z = z0
            while z != z1:
                P = P @ M[z]
                z = (z + 1) % 3
            return P

        full = [M[z] @ M[(z + 1) % 3] @ M[(z + 2) % 3] for z in range(3)]
        Z = np.trace(full[0])
        for zn in range(3):
            d = np.diag(full[zn])
            Cl = (self.S * d[:, None]).T @ self.S / Z  # (9, 9) same layer
            for p in range(9):
                for q in range(9):
                    C[p + 9 * zn, q + 9 * zn] = Cl[p, q]
        for zn in range(3):
            for zm in range(3):
                if zn == zm:
                    continue
                A = prod(zn, zm)
                B = prod(zm, zn)
                W = A * B.T
                Cl = self.S.T @ W @ self.S / Z
                for p in range(9):
                    for q in range(9):
                        C[p + 9 * zn, q + 9 * zm] = Cl[p, q]
        return C

    def mean_energy(self, beta: float, C: np.ndarray | None = None) -> float:
        if C is None:
            C = self.correlations(beta)
        L, N = 3, 27
        E = 0.0
        for site in range(N):
            x, y, z = site % 3, (site // 3) % 3, site // 9
            nbrs = [((x + 1) % 3) + 3 * (y + 3 * z), x + 3 * (((y + 1) % 3) + 3 * z),
                    x + 3 * (y + 3 * ((z + 1) % 3))]
            for d in range(3):
                E -= self.J[d * N + site] * C[site, nbrs[d]]
        return E

    def q2(self, beta: float, C: np.ndarray | None = None) -> float:
        if C is None:
            C = self.correlations(beta)
        return float((C ** 2).sum() / 27.0 ** 2)


def thermo_from_levels(g: np.ndarray, E: np.ndarray, beta: float):
    """(ln Z, <E>, var E) at beta from counts g[l] of states with energy E[l]."""
    mask = g > 0
    logw = np.log(g[mask].astype(np.float64)) - beta * E[mask]
    m = logw.max()
    w = np.exp(logw - m)
    Zs = w.sum()
    lnZ = m + math.log(Zs)
    Em = float((w * E[mask]).sum() / Zs)
    E2 = float((w * E[mask] ** 2).sum() / Zs)
    return lnZ, Em, E2 - Em * Em


__all__ = ["thermo_from_dos", "thermo_from_levels", "TransferMatrixL3", "density_of_states"]
