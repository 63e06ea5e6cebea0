"""Write l3_gauss_exact.json: exact thermodynamics of one L = 3 sample with
continuous Gaussian couplings (Sec. II.A), by two routes of the oracle.

Calls only the oracle: enumeration of all 2^27 states (oracle.r_exact_thermo:
ln Z, <E>, var E, ground-state energy) and the layer transfer matrix
(oracle.exact.TransferMatrixL3: ln Z, <E>), with the couplings of
pa_inputs.couplings_gauss (unit normals on the grid 2^-32) and beta F = -ln Z
(Eq. 9).

    python tests/golden/make_l3_gauss_exact.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import pa_inputs  # noqa: E402
from oracle.exact import TransferMatrixL3  # noqa: E402

COUPLING_SEED = 4321
BETAS = [0.0, 0.1, 0.2, 0.4, 0.6, 0.8, 1.0, 1.2, 1.4, 1.6, 1.8, 2.0, 3.0]


def main():
    oracle.build(force=False)
    J = pa_inputs.couplings_gauss(3, COUPLING_SEED)
    lnZ, Em, vE, E0 = oracle.r_exact_thermo(3, J, BETAS)
    tm = TransferMatrixL3(J)
    rows = []
    for k, b in enumerate(BETAS):
        rows.append(dict(beta=b, lnZ=float(lnZ[k]), mean_E=float(Em[k]), var_E=float(vE[k]),
                         lnZ_transfer=tm.lnZ(b), mean_E_transfer=tm.mean_energy(b)))
    out = dict(
        source="enumeration of 2^27 states (oracle.r_exact_thermo) and layer transfer matrix "
               "(oracle.exact.TransferMatrixL3)",
        model="3D Edwards-Anderson, L=3, periodic, Gaussian couplings on the grid 2^-32 "
              "(Sec. II.A); couplings pa_inputs.couplings_gauss",
        coupling_seed=COUPLING_SEED, E0=E0, sum_J2=float((J * J).sum()), rows=rows)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "l3_gauss_exact.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
