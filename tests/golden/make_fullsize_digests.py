"""Write tests/golden/fullsize_C3.json and fullsize_C2.json from the oracle.

    python tests/golden/make_fullsize_digests.py [C3] [C2]

Runs the CPU oracle (and nothing else) through the first steps of the two
full-size workloads defined in fullsize.py, with the synthetic couplings and
population seeds of pa_inputs, and stores per step: the FP64 scalars exactly,
the integer scalars, the digests of the copy counts, offsets, spins, energy
words and family labels, and (C2) both populations' overlap histogram.
About ten minutes of host time on eight cores for C3, one for C2.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import fullsize as fs  # noqa: E402
import oracle  # noqa: E402
import pa_inputs  # noqa: E402


def record(p, rec) -> dict:
    out = {k: float(getattr(rec, k)).hex() for k in fs.FLOATS}
    out.update({k: int(getattr(rec, k)) for k in fs.INTS})
    out["k"] = int(rec.k)
    out["counts"] = fs.u32_digest(p.last["n"])
    out["offsets"] = fs.u32_digest(p.last["offsets"])
    out["spins"] = fs.spins_digest(p.spins, p.R_tilde, p.N)
    out["U"] = fs.u32_digest(p.U[: p.R_tilde])
    out["family"] = fs.u32_digest(p.fam[: p.R_tilde])
    return out


def make_c3():
    w = fs.C3
    J = pa_inputs.couplings_pm(w["L"], pa_inputs.coupling_seed(w["config"], 0))
    seed = pa_inputs.population_seed(w["config"], 0, 0)
    p = oracle.Population(w["L"], J, w["R"], seed)
    steps = []
    for k in range(1, fs.C3_STEPS + 1):
        t0 = time.time()
        b = p.choose_beta(w["eps"], w["beta_max"])
        p.resample(b)
        p.sweep(b, w["n_sweeps"])
        steps.append(record(p, p.observables()))
        print(f"C3 step {k}: beta {b:.6f}, R~ {p.R_tilde}, {time.time() - t0:.1f} s", flush=True)
    return {"workload": w, "seed": seed, "steps": steps}


def make_c2():
    w = fs.C2
    J = pa_inputs.couplings_pm(w["L"], pa_inputs.coupling_seed(w["config"], 0))
    seeds = [pa_inputs.population_seed(w["config"], 0, pop) for pop in (0, 1)]
    pops = [oracle.Population(w["L"], J, w["R"], s) for s in seeds]
    betas = oracle.linear_schedule(w["beta_max"], w["n_temps"])
    steps = []
    for k in range(1, fs.C2_STEPS + 1):
        t0 = time.time()
        recs = []
        for p in pops:
            p.resample(betas[k])
            p.sweep(betas[k], w["n_sweeps"])
            recs.append(record(p, p.observables()))
        q, _ = oracle.overlap_hist(pops[0].N, pops[0].spins, pops[1].spins)
        steps.append({"pops": recs, "q": [int(x) for x in np.asarray(q)]})
        print(f"C2 step {k}: {time.time() - t0:.1f} s", flush=True)
    return {"workload": w, "seeds": seeds, "steps": steps}


def main():
    which = sys.argv[1:] or ["C3", "C2"]
    oracle.build(force=False)
    for name in which:
        data = {"C3": make_c3, "C2": make_c2}[name]()
        with open(fs.path(name), "w") as f:
            json.dump(data, f, indent=1)
        print("wrote", fs.path(name), flush=True)


if __name__ == "__main__":
    main()
