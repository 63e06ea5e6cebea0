"""Write l3_exact.json: exact thermodynamics of one L = 3 +-J sample.

Calls only the oracle's exact solvers (Gray-code enumeration of all 2^27
states for ln Z, <E>, var E; the layer transfer matrix for <q^2>), for the
3D Edwards-Anderson Hamiltonian of Sec. II.A with +-J couplings, the free
energy of Eq. 9 (beta F = -ln Z) and the spin overlap of Sec. II.A.

    python tests/golden/make_l3_exact.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import pa_inputs  # noqa: E402
from oracle.exact import TransferMatrixL3, thermo_from_dos  # noqa: E402

COUPLING_SEED = 1234
BETAS = [0.0, 0.05, 0.1, 0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 2.0, 3.0, 5.0]


def main():
    oracle.build(force=False)
    J = pa_inputs.couplings_pm(3, COUPLING_SEED)
    g = oracle.density_of_states(3, J)
    tm = TransferMatrixL3(J)
    rows = []
    for b in BETAS:
        lnZ, Em, vE = thermo_from_dos(g, 27, b)
        C = tm.correlations(b)
        rows.append(dict(beta=b, lnZ=lnZ, mean_E=Em, var_E=vE, q2=tm.q2(b, C),
                         lnZ_transfer=tm.lnZ(b), mean_E_transfer=tm.mean_energy(b, C)))
    out = dict(
        source="exact enumeration (2^27 states) and layer transfer matrix, oracle/exact.py",
        model="3D +-J Edwards-Anderson, L=3, periodic (Sec. II.A); couplings pa_inputs.couplings_pm",
        L=3, coupling_seed=COUPLING_SEED, dos=[int(x) for x in g], rows=rows)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "l3_exact.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
