"""Benchmark: population annealing at L=10, R=5e5 on one MI355X.

A step is one temperature step of the constant-culling anneal (Sec. III.C of
Amey & Machta, arXiv:1711.02146): choose beta' (bisection to a culling
fraction of 0.1), resample (histogram, FP64 table, copy counts, scan, copy
with family labels), 10 checkerboard Metropolis sweeps at beta', observables
(<E>, beta F, rho_t).  When the anneal reaches beta = 5 (about 190 steps
with +-J couplings, 210 with Gaussian ones) a new population starts again from
beta = 0 (its initialisation is timed too), so exactly --steps steps are timed;
the default 300 cover one whole anneal and the start of the next.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  value = spin-flip attempts per second of the whole
step loop (inputs resident in HBM), roofline = the sweep kernel (the dominant
kernel) timed with HIP events on its stream, cpu_baseline = the CPU oracle on
the first three steps of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = dict(name="L10_R500k_bitpack64_adaptive_eps0.1", L=10, R=500000, eps=0.1,
                beta_max=5.0, n_sweeps=10, layout="bitpack64", model="pm")
# The same anneal with Gaussian couplings quantised to 1/16 (reported beside
# the main line, not as its value).
GAUSS_WORKLOAD = dict(name="L10_R500k_bitpack64_gauss16_adaptive_eps0.1", L=10, R=500000,
                      eps=0.1, beta_max=5.0, n_sweeps=10, layout="bitpack64", model="gauss16")

# The same anneal with the couplings as real numbers (unit normals on the grid
# 2^-32): per-replica weights, exact fixed-point sums, the bisection on the device.
REAL_WORKLOAD = dict(name="L10_R500k_bitpack64_gauss_real_adaptive_eps0.1", L=10, R=500000,
                     eps=0.1, beta_max=5.0, n_sweeps=10, layout="bitpack64", model="gauss")

# Peak figures of one MI355X (gfx950): 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz
# retire 39.3e12 full-rate 32-bit VALU lane-instructions per second; HBM3E 8 TB/s.
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
# link overlap: per bond and pair, the XOR of the two ends' x words, the
# extraction of the pair's bit and its addition to the count
LINK_OPS_PER_BOND = 3
HBM_PEAK_GBS = 8000.0

# Algorithmic work of one spin-flip attempt, in gfx950 VALU lane-instructions
# (the unit of the peak above: one instruction per lane, whatever its number
# of inputs).  This count is fixed: it is the work of the bit-sliced algorithm
# below, and kernel changes that execute fewer instructions per attempt show as
# a higher fraction, never as a smaller count.
#   random number: a quarter of one Philox4x32-10 call, 10 rounds x (2
#   widening multiply-adds v_mad_u64_u32 + 2 three-input XORs v_bitop3) / 4 = 10;
#   +-J Metropolis test, bit-sliced: per site and 64 replicas, 6 J masks, 12
#   XORs (neighbour ^ own ^ J, two 32-replica halves), 16 adder instructions
#   (the bit planes of nu) and 68 to spread them into one byte per replica
#   (per half, 2 plane rotations, then 8 words x 3 masked merges and 1
#   rotation) = 102, i.e. 102/64 per attempt; per replica, the byte is the
#   threshold's address, then 1 compare (64-bit) and 1 select of the flip
#   mask's half = 2.
OPS_PER_ATTEMPT = 10 + 2 + 102 / 64
# Gaussian couplings, bit-sliced pattern pass: per site and 64 replicas, 12
# XORs (neighbour ^ own, two 32-replica halves) and 120 to spread the six
# "neighbour differs" planes into one byte per replica holding 4 y (per half,
# 5 plane rotations, then 8 words x (1 AND + 5 masked merges) and 7 rotations)
# = 132, i.e. 132/64 per attempt.  Per replica, quantised couplings (k = 16 J):
# the byte is the offset of the site's table entry, whose value is the LDS
# address of the dE16 threshold, then 1 compare (64-bit) and 1 select of the
# flip mask's half = 2; real couplings: the byte is the offset of the site's
# 4-byte entry min(thr, 2^32 - 1), then 1 compare (32-bit), 1 select, and 1 for
# the search of the draw 2^32 - 1 among each lane's four draws (3 max + 1
# compare per four), where the exact 8-byte threshold decides = 3.  Each site
# and wave also reads one table row through the caches (a 64-lane gather).
OPS_PER_ATTEMPT_GAUSS = 10 + 2 + 132 / 64
OPS_PER_ATTEMPT_REAL = 10 + 3 + 132 / 64
# Algorithmic HBM bytes of one sweep launch: the bit-packed population read and
# written once (N bits per replica each way) plus 20 B per replica (source index,
# energy and family label read, energy and family label written).
BYTES_PER_REPLICA_FIXED = 20

# Counters of the sweep kernel from rocprofv3 on this workload, per launch,
# with the kernel source they were taken on (reported only while that source
# is unchanged): HBM bytes = FETCH_SIZE x 2 + WRITE_SIZE x 1 (the factors a
# plain copy of known size reads, --copy-calibration), and the executed VALU
# lane-instructions per attempt = SQ_INSTS_VALU x 64 / attempts per launch.
# None: no counters for the current source yet.
PROFILE = {
    "kernel_src_sha256": "09a636d0398f288f2ffcc9e73ed17ebb9a9070905e5d048eb50c82aaedef6373",
    # FETCH_SIZE KiB x 2 + WRITE_SIZE KiB x 1, per launch (profiles/*_hbm_counters.md)
    "bytes_per_launch": (32861.6 * 2 + 64946.1) * 1024,
    "gauss16_bytes_per_launch": (33336.6 * 2 + 64942.5) * 1024,
    "real_bytes_per_launch": (35163.6 * 2 + 66898.5) * 1024,
    "link_overlap_bytes_per_launch": (61563.2 * 2 + 10484.4) * 1024,
    "int8_C2_bytes_per_launch": (26059.5 * 2 + 50797.2) * 1024,
    "int8_overlap_bytes_per_call": (50034.2 * 2 + 342.9) * 1024,
    # SQ_INSTS_VALU 1.0286e9 per launch x 64 lanes / 5.0e9 attempts
    "valu_per_attempt": 1.0286e9 * 64 / 5.0e9,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-instance batch run")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the built-in sweep-form rule instead of timing both forms first")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="arrival window of the serving run (0 skips it)")
    ap.add_argument("--serve-only", action="store_true",
                    help="only run the serving workload and print its JSON object")
    ap.add_argument("--serve-max-active", type=int, default=0,
                    help="resident-request limit of the serving run (default 256)")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="request rate of the serving run (default 4 per second)")
    ap.add_argument("--serve-load-seconds", type=float, default=15.0,
                    help="arrival window of a second serving run at --serve-load-rate, which "
                         "keeps several requests resident at once (0 skips it)")
    ap.add_argument("--serve-load-rate", type=float, default=24.0,
                    help="request rate of that run")
    ap.add_argument("--serve-lockstep", action="store_true",
                    help="step every resident request on every tick (no work-fair selection)")
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--gauss-steps", type=int, default=300,
                    help="timed steps of the Gaussian-coupling anneal (0 skips it)")
    ap.add_argument("--no-int8", action="store_true", help="skip the int8-layout C1/C2 runs")
    ap.add_argument("--real-steps", type=int, default=50,
                    help="steps of the real-Gaussian-coupling anneal (0: skip)")
    ap.add_argument("--oracle-one-thread", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 5 times (used to "
                         "scale the HBM byte counters of a profiler run)")
    return ap.parse_args()


def copy_calibration(nbytes: int):
    import torch

    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 5}), flush=True)


def event_pairs(n):
    """n pairs of timing events, each recorded once so that its HIP event
    exists before a timed region (torch creates it at the first record)."""
    import torch

    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
             for _ in range(n)]
    for e0, e1 in pairs:
        e0.record()
        e1.record()
    torch.cuda.synchronize()
    return pairs


def run_steps(pam, J, w, n_steps, seed0, sweeps=None, stats=None, anneals=None):
    """n_steps temperature steps of the constant-culling anneal (step choice,
    resample, sweeps, observables), taken with pa_anneal_run: many steps per
    call, one synchronisation per step, the family sums of one step computed
    on the device while the host chooses the next; a new population at beta = 0
    whenever beta_max is hit.  sweeps (list, optional) receives (sweep launch
    ms, R~) per step: the library brackets each sweep launch with HIP events on
    the population's stream (PA_FLAG_TIME_SWEEPS); anneals (list, optional)
    receives the step count of every anneal completed."""
    attempts = 0
    pop = None
    gen = 0
    in_anneal = 0
    flags = pam.PA_FLAG_TIME_SWEEPS if sweeps is not None else 0
    N = w["L"] ** 3
    left = n_steps
    while left > 0:
        if pop is None or pop_beta >= w["beta_max"]:
            if pop is not None:
                pop.close()
                if anneals is not None:
                    anneals.append(in_anneal)
            pop = pam.Population(w["L"], w["R"], J, seed0 + gen, layout=w["layout"],
                                 model=w["model"], flags=flags)
            pop_beta = 0.0
            in_anneal = 0
            gen += 1
        chunk = pop.anneal_run(w["eps"], w["beta_max"], w["n_sweeps"], left)
        for obs in chunk:
            attempts += w["n_sweeps"] * N * obs["R_tilde"]
            if sweeps is not None:
                sweeps.append((obs["sweep_ms"], obs["R_tilde"]))
            if stats is not None:
                stats.append((obs["beta"], obs["R_tilde"], obs["rho_t"], obs["beta_F"]))
        pop_beta = chunk[-1]["beta"]
        in_anneal += len(chunk)
        left -= len(chunk)
    if pop is not None:
        pop.close()
        if anneals is not None and pop_beta >= w["beta_max"]:
            anneals.append(in_anneal)
    return attempts


def whole_anneal(pam, J, w, seed):
    """One complete anneal from a new population at beta = 0 to beta_max, timed
    from creation (initialisation included) to the last step's observables."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pop = pam.Population(w["L"], w["R"], J, seed, layout=w["layout"], model=w["model"])
    chunk = pop.anneal_run(w["eps"], w["beta_max"], w["n_sweeps"], 100000)
    steps = len(chunk)
    attempts = sum(w["n_sweeps"] * w["L"] ** 3 * o["R_tilde"] for o in chunk)
    obs = chunk[-1]
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out = {"steps": steps, "seconds": round(t, 4), "attempts": attempts,
           "attempts_per_s": attempts / t, "beta_F": obs["beta_F"], "rho_t": obs["rho_t"],
           "E_min": obs["E_min"]}
    pop.close()
    return out


def copy_rate_GBs(nbytes: int = 1 << 30, repeats: int = 5) -> float:
    """Sustained device-to-device copy rate (read + write bytes per second) of a
    plain torch copy of nbytes, timed with HIP events: the measured HBM ceiling."""
    import torch

    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ms = []
    for e0, e1 in event_pairs(repeats):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (min(ms) * 1e-3) / 1e9


BATCH = dict(name="256_instances_L4-10_R2e4-1e5_2pops_NT101_NS10", n_instances=256, Ls=(4, 6, 8, 10),
             R_lo=20000, R_hi=100000, n_temps=101, beta_max=5.0, n_sweeps=10, sample_every=16)


def batch_instances(c):
    """The 256 synthetic instances: (L, R, couplings, seed A, seed B), seeded."""
    import numpy as np

    import pa_inputs

    rng = np.random.Generator(np.random.PCG64(0xBA7C4))
    out = []
    for i in range(c["n_instances"]):
        L = int(rng.choice(c["Ls"]))
        R = int(rng.integers(c["R_lo"], c["R_hi"] + 1))
        J = pa_inputs.couplings_pm(L, pa_inputs.coupling_seed(4, i))
        out.append((L, R, J, pa_inputs.population_seed(4, i, 0), pa_inputs.population_seed(4, i, 1)))
    return out


def size_class(R: int) -> int:
    """floor(log2(ceil(R / 64))): the autotuner's size class of a population."""
    return ((R + 63) // 64).bit_length() - 1


def layout_tune(pam, L, R, J, seed, beta=0.3, n_sweeps=10, repeats=3):
    """Time both spin layouts on (L, R) and record the faster for "auto"."""
    t = pam.pa_autotune_layout(L, R, J, seed=seed, beta=beta, n_sweeps=n_sweeps, repeats=repeats)
    return {"L": L, "R": R, "size_class": size_class(R), "layout": t["layout"],
            "ms_int8": t["ms_int8"], "ms_bitpack64": t["ms_bitpack64"]}


def batched_bench(pam, layout="auto"):
    """All instances in one batch (one graph replay per step) against back-to-back
    single-instance runs of every sample_every-th instance, extrapolated.  With
    layout "auto" the layout autotuner first times both layouts on each
    (L, size class) the instances fall into; every population then takes the
    faster (batch and back-to-back runs alike)."""
    import numpy as np
    import torch

    c = BATCH
    insts = batch_instances(c)
    tuned = []
    if layout == "auto":
        seen = set()
        for (L, R, J, sa, _sb) in insts:
            if (L, size_class(R)) not in seen:
                seen.add((L, size_class(R)))
                tuned.append(layout_tune(pam, L, R, J, sa, beta=1.0, n_sweeps=c["n_sweeps"]))
    layouts_used = {}
    for (L, R, *_r) in insts:
        lay = pam.pa_layout_choice(L, R) if layout == "auto" else layout
        layouts_used.setdefault(str(L), {}).setdefault(lay, 0)
        layouts_used[str(L)][lay] += 1
    betas = pam.linear_schedule(c["beta_max"], c["n_temps"])
    n_steps = len(betas) - 1
    attempts = sum(2 * n_steps * c["n_sweeps"] * L ** 3 * R for (L, R, *_r) in insts)
    # batched: creation (init of every population, graph capture) + all steps + results
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pops = []
    for (L, R, J, sa, sb) in insts:
        pops.append(pam.Population(L, R, J, sa, layout=layout, stream=stream))
        pops.append(pam.Population(L, R, J, sb, layout=layout, stream=stream))
    b = pam.Batch(pops, betas, c["n_sweeps"], pairs=[(2 * i, 2 * i + 1) for i in range(len(insts))])
    t1 = time.perf_counter()
    b.run()
    recs, q, status = b.results()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    b.close()
    for p in pops:
        p.close()
    del pops
    torch.cuda.empty_cache()
    t_batch = t2 - t0
    # back to back: the same calls one instance at a time, default stream
    sample = list(range(0, len(insts), c["sample_every"]))
    identical = True
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for i in sample:
        L, R, J, sa, sb = insts[i]
        pa_ = pam.Population(L, R, J, sa, layout=layout)
        pb_ = pam.Population(L, R, J, sb, layout=layout)
        for k in range(1, len(betas)):
            for pidx, p in ((2 * i, pa_), (2 * i + 1, pb_)):
                p.resample(betas[k])
                p.sweep(betas[k], c["n_sweeps"])
                o = p.observables()
                r = recs[k - 1][pidx]
                identical &= (o["beta_F"] == r["beta_F"] and o["mean_E"] == r["mean_E"]
                              and o["rho_t"] == r["rho_t"] and o["R_tilde"] == r["R_tilde"])
            h = pam.overlap_hist(pa_, pb_)
            identical &= bool(np.array_equal(h, q[k - 1][i]))
        pa_.close()
        pb_.close()
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    t_single = (t4 - t3) * len(insts) / len(sample)
    return {
        "workload": c["name"],
        "instances": len(insts),
        "populations": 2 * len(insts),
        "steps": n_steps,
        "attempts": attempts,
        "batched_seconds": round(t_batch, 3),
        "batched_setup_seconds": round(t1 - t0, 3),
        "batched_instances_per_hour": len(insts) * 3600.0 / t_batch,
        "batched_attempts_per_s": attempts / t_batch,
        "back_to_back_seconds_extrapolated": round(t_single, 3),
        "back_to_back_instances_per_hour": len(insts) * 3600.0 / t_single,
        "back_to_back_sample": f"{len(sample)} of {len(insts)} instances (every {c['sample_every']}th)",
        "speedup": t_single / t_batch,
        "identical_on_sample": bool(identical),
        "capacity_failures": int(np.count_nonzero(status)),
        "layout": layout,
        # instances per L in each layout, and the autotuner's timings per
        # (L, size class): best sweep launch of n_sweeps sweeps at beta = 1
        "layouts_per_L": layouts_used,
        "layout_autotune": tuned,
    }


SERVE = dict(name="poisson4_L4-12_R1e4-2e5_loguniform_NT51-201_NS10", rate=4.0, beta_max=5.0,
             n_sweeps=10, hbm_budget=64 << 30, max_active=256, max_L=12)


def serving_bench(duration_s: float, max_active: int | None = None, rate: float | None = None,
                  fair: bool = True):
    """Poisson request stream served with continuous batching (real time)."""
    import numpy as np

    import pa_inputs
    from paper_1711_02146_amd.serve import Request, Server

    c = SERVE
    rate = rate or c["rate"]
    specs = pa_inputs.serving_requests(duration_s=duration_s, rate=rate)
    reqs = [Request(rid=d["rid"], arrival=d["arrival"], L=d["L"], R=d["R"], n_temps=d["n_temps"],
                    n_sweeps=c["n_sweeps"], beta_max=c["beta_max"],
                    J=pa_inputs.couplings_pm(d["L"], d["coupling_seed"]), seed=d["seed"])
            for d in specs]
    srv = Server(hbm_budget=c["hbm_budget"], max_active=max_active or c["max_active"],
                 max_L=c["max_L"], fair=fair)
    last = [time.perf_counter()]

    def progress(t, done, active, queued):
        if time.perf_counter() - last[0] > 10.0:
            last[0] = time.perf_counter()
            print(f"# serve t={t:.0f}s done={done} active={active} queued={queued}",
                  file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    res = srv.run(reqs, realtime=True, progress=progress)
    wall = time.perf_counter() - t0
    srv.close()
    ok = [r for r in res if r.status == 0]
    lat = np.array([r.latency for r in ok])
    att = sum(r.attempts for r in ok)
    span = max(r.finished for r in ok) - min(r.arrival for r in ok)
    sizes = np.array(srv.tick_sizes)
    return {
        "workload": c["name"] if rate == c["rate"] else c["name"].replace("poisson4", f"poisson{rate:g}"),
        "rate_per_s": rate,
        "tick_policy": "work-fair" if fair else "every resident each tick",
        "arrival_seconds": duration_s,
        "requests": len(reqs),
        "completed": len(ok),
        "failed": len(res) - len(ok),
        "offered_attempts_per_s": sum(r.attempts() for r in reqs) / duration_s,
        "attempts_per_s": att / span,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(lat.max()),
        "ticks": srv.ticks,
        "mean_resident": float(sizes.mean()) if sizes.size else 0.0,
        "max_resident": int(sizes.max()) if sizes.size else 0,
        "max_active": max_active or c["max_active"],
        "hbm_budget_bytes": c["hbm_budget"],
        "wall_seconds": wall,
    }


def sweep_roofline(w, sweeps, ops_per_attempt, layout_bytes_per_site):
    """Average sweep launch of a timed run against the VALU peak.
    sweeps: (ms, R~) per launch; layout_bytes_per_site: spin bytes per site and
    replica in HBM (1/8 bit-packed, 1 int8)."""
    sweep_ms = [ms for ms, _ in sweeps]
    sweep_att = sum(w["n_sweeps"] * w["L"] ** 3 * r for _, r in sweeps)
    n_launch = len(sweep_ms)
    avg_ms = sum(sweep_ms) / n_launch
    avg_att = sweep_att / n_launch
    achieved_ops = ops_per_attempt * avg_att / (avg_ms * 1e-3)
    avg_R = avg_att / (w["n_sweeps"] * w["L"] ** 3)
    bytes_per_launch = (2 * avg_R * w["L"] ** 3 * layout_bytes_per_site
                        + BYTES_PER_REPLICA_FIXED * avg_R)
    return dict(sweep_ms=sweep_ms, avg_ms=avg_ms, avg_att=avg_att, n_launch=n_launch,
                achieved_ops=achieved_ops, bytes_per_launch=bytes_per_launch)


C1 = dict(name="C1_L4_R1000_int8_linear_NT51_NS10", L=4, R=1000, n_temps=51, beta_max=5.0,
          n_sweeps=10, layout="int8", config=1)
C2 = dict(name="C2_L8_R1e5_int8_2pops_linear_NT201_NS10_q65", L=8, R=100000, n_temps=201,
          beta_max=5.0, n_sweeps=10, layout="int8", config=2)


def linear_run(pam, c, pops_n, with_q):
    """A whole linear-schedule run of the config: pops_n populations of one
    sample stepped in lockstep (one pa_anneal_step each per temperature), the
    overlap histogram of the first two after every step when with_q.  Timed
    from the creation of the populations to the last result."""
    import numpy as np
    import torch

    import pa_inputs

    J = pa_inputs.couplings_pm(c["L"], pa_inputs.coupling_seed(c["config"], 0))
    seeds = [pa_inputs.population_seed(c["config"], 0, p) for p in range(pops_n)]
    betas = pam.linear_schedule(c["beta_max"], c["n_temps"])
    N = c["L"] ** 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pops = [pam.Population(c["L"], c["R"], J, s, layout=c["layout"],
                           flags=pam.PA_FLAG_TIME_SWEEPS) for s in seeds]
    attempts, sweep_ms, sweep_att, q_ms, last = 0, [], 0, [], None
    for k in range(1, len(betas)):
        for p in pops:
            o = p.step_to(betas[k], c["n_sweeps"])
            attempts += c["n_sweeps"] * N * o["R_tilde"]
            sweep_ms.append(o["sweep_ms"])
            sweep_att += c["n_sweeps"] * N * o["R_tilde"]
            last = o
        if with_q:
            t1 = time.perf_counter()
            q = pam.overlap_hist(pops[0], pops[1])
            q_ms.append(1e3 * (time.perf_counter() - t1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avg_ms = sum(sweep_ms) / len(sweep_ms)
    avg_att = sweep_att / len(sweep_ms)
    avg_R = avg_att / (c["n_sweeps"] * N)
    profiled = PROFILE is not None and PROFILE["kernel_src_sha256"] == kernel_src_sha256()
    ops = OPS_PER_ATTEMPT * avg_att / (avg_ms * 1e-3)
    bytes_launch = 2 * avg_R * N + BYTES_PER_REPLICA_FIXED * avg_R
    out = {"workload": c["name"], "populations": pops_n, "steps": len(betas) - 1,
           "attempts": attempts, "seconds": round(wall, 4), "value": attempts / wall,
           "unit": "attempts/s",
           "sweep": {"kernel": f"k_sweep<int8, L={c['L']}, +-J>", "avg_launch_ms": avg_ms,
                     "launches": len(sweep_ms), "attempts_per_launch": avg_att,
                     "sweep_attempts_per_s": avg_att / (avg_ms * 1e-3),
                     "bound": "alu", "achieved": ops / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": ops / VALU_PEAK_OPS,
                     "ops_per_attempt": OPS_PER_ATTEMPT,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "hbm_algorithmic_GBs": bytes_launch / (avg_ms * 1e-3) / 1e9,
                     "bytes_per_attempt": bytes_launch / avg_att,
                     # rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE per launch (C2's shape only)
                     "traffic": (PROFILE["int8_C2_bytes_per_launch"]
                                 if profiled and c["config"] == 2 else None)},
           "beta_F": [p.observables()["beta_F"] for p in pops], "rho_t": last["rho_t"]}
    if with_q:
        pairs = min(p.observables()["R_tilde"] for p in pops[:2])
        out["overlap"] = {"kernel": "k_overlap<int8> (+ clear, copy of 65 counts, sync)",
                          "avg_call_ms": sum(q_ms) / len(q_ms), "calls": len(q_ms),
                          "pairs": pairs, "algorithmic_bytes": 2 * pairs * N,
                          "hbm_GBs": 2 * pairs * N / (sum(q_ms) / len(q_ms) * 1e-3) / 1e9,
                          "kernel_traffic": (PROFILE["int8_overlap_bytes_per_call"]
                                             if profiled else None),
                          "q_bins_nonzero": int(np.count_nonzero(q))}
    for p in pops:
        p.close()
    return out


def int8_cpu_baseline(c, pops_n, with_q, n_steps):
    """The oracle on the first n_steps of the int8 config (all of C1)."""
    import oracle
    import pa_inputs

    oracle.build(force=False)
    J = pa_inputs.couplings_pm(c["L"], pa_inputs.coupling_seed(c["config"], 0))
    betas = oracle.linear_schedule(c["beta_max"], c["n_temps"])
    t0 = time.perf_counter()
    pops = [oracle.Population(c["L"], J, c["R"], pa_inputs.population_seed(c["config"], 0, p))
            for p in range(pops_n)]
    att = 0
    for k in range(1, n_steps + 1):
        for p in pops:
            p.resample(betas[k])
            p.sweep(betas[k], c["n_sweeps"])
            p.observables()
            att += c["n_sweeps"] * c["L"] ** 3 * p.R_tilde
        if with_q:
            oracle.overlap_hist(pops[0].N, pops[0].spins, pops[1].spins)
    t = time.perf_counter() - t0
    return {"value": att / t, "unit": "attempts/s", "cores": omp_threads(), "kind": "oracle",
            "sample": f"the first {n_steps} of {len(betas) - 1} steps" if n_steps < len(betas) - 1
                      else "the whole run", "seconds": round(t, 2)}


def gauss_bench(pam, steps: int, warmup: int, autotune: bool):
    """The benchmark anneal with quantised Gaussian couplings (k = 16 J)."""
    import torch

    import pa_inputs

    w = GAUSS_WORKLOAD
    K = pa_inputs.couplings_gauss16(w["L"], pa_inputs.coupling_seed(3, 0))
    seed0 = pa_inputs.population_seed(3, 0, 0)
    tune = None
    if autotune:
        tp = pam.Population(w["L"], w["R"], K, seed0 + 999, layout=w["layout"], model=w["model"])
        tune = tp.autotune(beta=0.3, n_sweeps=w["n_sweeps"], repeats=5)
        tp.close()
    run_steps(pam, K, w, warmup, seed0 + 1000)
    sweeps, stats, anneals = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    attempts = run_steps(pam, K, w, steps, seed0, sweeps, stats, anneals)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r = sweep_roofline(w, sweeps, OPS_PER_ATTEMPT_GAUSS, 1 / 8)
    link = link_overlap_bench(pam, K, w)
    traffic = None
    if PROFILE is not None and PROFILE["kernel_src_sha256"] == kernel_src_sha256():
        traffic = PROFILE["gauss16_bytes_per_launch"]
        link["traffic"] = PROFILE["link_overlap_bytes_per_launch"]
    return {
        "workload": w["name"], "couplings": "Gaussian N(0,1) rounded to 1/16, k in [-127, 127]",
        "value": attempts / wall, "unit": "attempts/s", "steps": steps, "warmup": warmup,
        "ms_per_step": 1e3 * wall / steps,
        "sweep": {"kernel": "k_sweep<bitpack64, L=10, gauss16> (gather + 10 sweeps + energy)",
                  "avg_launch_ms": r["avg_ms"], "launches": r["n_launch"],
                  "attempts_per_launch": r["avg_att"],
                  "sweep_attempts_per_s": r["avg_att"] / (r["avg_ms"] * 1e-3),
                  "achieved": r["achieved_ops"] / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                  "unit": "Tops/s", "frac": r["achieved_ops"] / VALU_PEAK_OPS,
                  "ops_per_attempt": OPS_PER_ATTEMPT_GAUSS,
                  "traffic": traffic, "algorithmic_bytes_per_launch": r["bytes_per_launch"],
                  "hbm_algorithmic_GBs": r["bytes_per_launch"] / (r["avg_ms"] * 1e-3) / 1e9},
        "sweep_fraction_of_wall": sum(r["sweep_ms"]) * 1e-3 / wall,
        "autotune": tune,
        "anneals_completed": len(anneals),
        "steps_per_anneal": anneals,
        "beta_at_end": stats[-1][0] if stats else None,
        "link_overlap": link,
    }


def gauss_real_bench(pam, steps: int, warmup: int, autotune: bool):
    """The benchmark anneal with real Gaussian couplings (PA_MODEL_GAUSS)."""
    import torch

    import pa_inputs

    w = REAL_WORKLOAD
    J = pa_inputs.couplings_gauss(w["L"], pa_inputs.coupling_seed(3, 0))
    seed0 = pa_inputs.population_seed(3, 0, 0)
    tune = None
    if autotune:
        tp = pam.Population(w["L"], w["R"], J, seed0 + 999, layout=w["layout"], model=w["model"])
        tune = tp.autotune(beta=0.3, n_sweeps=w["n_sweeps"], repeats=5)
        tp.close()
    run_steps(pam, J, w, warmup, seed0 + 1000)
    sweeps, stats, anneals = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    attempts = run_steps(pam, J, w, steps, seed0, sweeps, stats, anneals)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r = sweep_roofline(w, sweeps, OPS_PER_ATTEMPT_REAL, 1 / 8)
    return {
        "workload": w["name"],
        "couplings": "Gaussian N(0,1) as FP64 on the grid 2^-32 (int64 energy words)",
        "value": attempts / wall, "unit": "attempts/s", "steps": steps, "warmup": warmup,
        "ms_per_step": 1e3 * wall / steps,
        "sweep": {"kernel": "k_sweep<bitpack64, L=10, real> (gather + 10 sweeps + energy)",
                  "avg_launch_ms": r["avg_ms"], "launches": r["n_launch"],
                  "attempts_per_launch": r["avg_att"],
                  "sweep_attempts_per_s": r["avg_att"] / (r["avg_ms"] * 1e-3),
                  "achieved": r["achieved_ops"] / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                  "unit": "Tops/s", "frac": r["achieved_ops"] / VALU_PEAK_OPS,
                  "ops_per_attempt": OPS_PER_ATTEMPT_REAL,
                  "traffic": (PROFILE["real_bytes_per_launch"] if PROFILE is not None and
                              PROFILE["kernel_src_sha256"] == kernel_src_sha256() else None),
                  "algorithmic_bytes_per_launch": r["bytes_per_launch"],
                  "hbm_algorithmic_GBs": r["bytes_per_launch"] / (r["avg_ms"] * 1e-3) / 1e9},
        "sweep_fraction_of_wall": sum(r["sweep_ms"]) * 1e-3 / wall,
        "outside_sweep_us_per_step": 1e6 * (wall - sum(r["sweep_ms"]) * 1e-3) / steps,
        "autotune": tune,
        "anneals_completed": len(anneals),
        "steps_per_anneal": anneals,
        "beta_at_end": stats[-1][0] if stats else None,
    }


def gauss_real_cpu_baseline(w, R_sample=50000, n_steps=2):
    """The oracle on the first n_steps temperature steps of the real-coupling
    workload at a tenth of its population (same L, couplings and culling)."""
    import oracle
    import pa_inputs

    oracle.build(force=False)
    J = pa_inputs.couplings_gauss(w["L"], pa_inputs.coupling_seed(3, 0))
    t0 = time.perf_counter()
    p = oracle.GaussRealPopulation(w["L"], J, R_sample, pa_inputs.population_seed(3, 0, 0))
    att = 0
    for _ in range(n_steps):
        b = p.choose_beta(w["eps"], w["beta_max"])
        p.resample(b)
        p.sweep(b, w["n_sweeps"])
        p.observables()
        att += w["n_sweeps"] * w["L"] ** 3 * p.R_tilde
    t1 = time.perf_counter()
    return {"value": att / (t1 - t0), "unit": "attempts/s", "cores": omp_threads(), "kind": "oracle",
            "sample": f"the first {n_steps} temperature steps (init, then step choice + resample + "
                      f"{w['n_sweeps']} sweeps each) of the real-coupling workload at R={R_sample}",
            "seconds": round(t1 - t0, 2)}


def link_overlap_bench(pam, K, w, repeats: int = 5):
    """The link-overlap histogram (Sec. II.A q_l) between two independent
    populations of the Gaussian workload's size after N_S sweeps at beta = 0.3:
    HIP events on the populations' stream around each call (the call clears
    the partial counts, runs k_link_overlap and k_link_reduce, and copies the
    3N + 1 counts back)."""
    import numpy as np

    import pa_inputs

    seed = pa_inputs.population_seed(3, 0, 1)
    a = pam.Population(w["L"], w["R"], K, seed, layout=w["layout"], model=w["model"])
    b = pam.Population(w["L"], w["R"], K, seed + 1, layout=w["layout"], model=w["model"])
    for p in (a, b):
        p.sweep(0.3, w["n_sweeps"])
    pam.link_overlap_hist(a, b)
    ms = []
    for e0, e1 in event_pairs(repeats):
        e0.record(a.stream)
        h = pam.link_overlap_hist(a, b)
        e1.record(a.stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    pairs = int(h.sum())
    N = w["L"] ** 3
    q_l = float(1.0 - 2.0 * (h * np.arange(h.size)).sum() / (pairs * 3 * N))
    a.close()
    b.close()
    avg = sum(ms) / len(ms)
    ops = LINK_OPS_PER_BOND * 3 * N * pairs
    return {"kernel": "k_link_overlap<bitpack64> (one 64-pair tile per wave)", "pairs": pairs,
            "avg_call_ms": avg, "pairs_per_s": pairs / (avg * 1e-3),
            "ops_per_bond": LINK_OPS_PER_BOND, "achieved": ops / (avg * 1e-3) / 1e12,
            "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s",
            "frac": ops / (avg * 1e-3) / VALU_PEAK_OPS,
            "algorithmic_bytes": 2 * pairs * N // 8, "traffic": None, "q_l_mean": q_l,
            "beta": 0.3}


def gauss_cpu_baseline(w, R_sample=100000, n_steps=3):
    """The oracle on the first n_steps temperature steps of the Gaussian-coupling
    workload at a fifth of its population (same L, couplings and culling)."""
    import oracle
    import pa_inputs

    oracle.build(force=False)
    K = pa_inputs.couplings_gauss16(w["L"], pa_inputs.coupling_seed(3, 0))
    t0 = time.perf_counter()
    p = oracle.GaussPopulation(w["L"], K, R_sample, pa_inputs.population_seed(3, 0, 0))
    att = 0
    for _ in range(n_steps):
        b = p.choose_beta(w["eps"], w["beta_max"])
        p.resample(b)
        p.sweep(b, w["n_sweeps"])
        p.observables()
        att += w["n_sweeps"] * w["L"] ** 3 * p.R_tilde
    t1 = time.perf_counter()
    return {"value": att / (t1 - t0), "unit": "attempts/s", "cores": omp_threads(), "kind": "oracle",
            "sample": f"the first {n_steps} temperature steps (init, then step choice + resample + "
                      f"{w['n_sweeps']} sweeps each) of the Gaussian workload at R={R_sample}",
            "seconds": round(t1 - t0, 2)}


def kernel_src_sha256():
    """SHA-256 over the kernel sources (pa_kernels.hip and the file it includes)."""
    import hashlib

    h = hashlib.sha256()
    for name in ("pa_kernels.hip", "pa_real_kernels.inc", "pa_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1711_02146_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def omp_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_steps=3):
    """The oracle on the first n_steps temperature steps of the same workload
    (initialisation included), on all host threads; and on one thread (a child
    process with OMP_NUM_THREADS=1) over the first step at a fifth of R."""
    import subprocess

    import oracle
    import pa_inputs

    oracle.build(force=False)
    J = pa_inputs.couplings_pm(w["L"], pa_inputs.coupling_seed(3, 0))
    t0 = time.perf_counter()
    p = oracle.Population(w["L"], J, w["R"], pa_inputs.population_seed(3, 0, 0))
    att, t_sweep = 0, 0.0
    for _ in range(n_steps):
        b = p.choose_beta(w["eps"], w["beta_max"])
        p.resample(b)
        t1 = time.perf_counter()
        p.sweep(b, w["n_sweeps"])
        t_sweep += time.perf_counter() - t1
        p.observables()
        att += w["n_sweeps"] * w["L"] ** 3 * p.R_tilde
    t2 = time.perf_counter()
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-one-thread"],
                         env=env, capture_output=True, text=True, check=True)
    return {"value": att / (t2 - t0), "unit": "attempts/s", "cores": omp_threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"the first {n_steps} temperature steps (init, then step choice + resample + "
                      f"{w['n_sweeps']} sweeps each, {att:.3g} attempts) of the same workload; "
                      f"sweeps alone {att / t_sweep:.3g} attempts/s",
            "seconds": round(t2 - t0, 2),
            "one_thread": json.loads(one.stdout.strip().splitlines()[-1])}


def oracle_one_thread(w=None, R_sample=100000):
    """Run in a child with OMP_NUM_THREADS=1: the oracle on the first step of
    the workload at R_sample replicas (same L, couplings and culling)."""
    import oracle
    import pa_inputs

    w = w or WORKLOAD
    oracle.build(force=False)
    J = pa_inputs.couplings_pm(w["L"], pa_inputs.coupling_seed(3, 0))
    t0 = time.perf_counter()
    p = oracle.Population(w["L"], J, R_sample, pa_inputs.population_seed(3, 0, 0))
    b = p.choose_beta(w["eps"], w["beta_max"])
    p.resample(b)
    p.sweep(b, w["n_sweeps"])
    p.observables()
    t = time.perf_counter() - t0
    att = w["n_sweeps"] * w["L"] ** 3 * p.R_tilde
    print(json.dumps({"value": att / t, "unit": "attempts/s", "cores": 1, "kind": "oracle",
                      "sample": f"the first temperature step at R={R_sample} ({att:.3g} attempts)",
                      "seconds": round(t, 2)}), flush=True)


def main():
    args = parse()
    if args.oracle_one_thread:
        oracle_one_thread()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no "
              "multi-GPU path; value is one GPU's throughput.", file=sys.stderr)
        sys.exit(2)
    import torch

    import pa_inputs
    import paper_1711_02146_amd as pam

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    pam.lib()
    if args.serve_only:
        print(json.dumps({"serving": serving_bench(args.serve_seconds,
                                                   args.serve_max_active or None,
                                                   args.serve_rate or None,
                                                   not args.serve_lockstep)}), flush=True)
        return
    w = WORKLOAD
    J = pa_inputs.couplings_pm(w["L"], pa_inputs.coupling_seed(3, 0))
    seed0 = pa_inputs.population_seed(3, 0, 0)
    print(f"# warmup {args.warmup} steps (and the sweep autotuner on this shape)", file=sys.stderr,
          flush=True)
    tune, ltune = None, None
    if not args.no_autotune:
        # spin layout first (each timed in its faster sweep form), then the
        # sweep form of the chosen layout on its own population
        ltune = layout_tune(pam, w["L"], w["R"], J, seed0 + 998, n_sweeps=w["n_sweeps"],
                            repeats=5)
        w = dict(w, layout=ltune["layout"], name=w["name"].replace("bitpack64", ltune["layout"]))
        tp = pam.Population(w["L"], w["R"], J, seed0 + 999, layout=w["layout"])
        # tuned at beta = 0.3, the middle of the temperatures the timed steps cover
        tune = tp.autotune(beta=0.3, n_sweeps=w["n_sweeps"], repeats=5)
        tp.close()
    run_steps(pam, J, w, args.warmup, seed0 + 1000)
    # this device's measured ceilings: sustained VALU issue, Philox draws alone,
    # and the plain copy rate of HBM
    ceil = pam.pa_probe_ceilings()
    copy_GBs = copy_rate_GBs()
    torch.cuda.synchronize()
    print(f"# timing {args.steps} steps", file=sys.stderr, flush=True)
    sweeps, stats, anneals = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    attempts = run_steps(pam, J, w, args.steps, seed0, sweeps, stats, anneals)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    r = sweep_roofline(w, sweeps, OPS_PER_ATTEMPT, 1 / 8 if w["layout"] == "bitpack64" else 1.0)
    sweep_ms, avg_ms, avg_att, n_launch = r["sweep_ms"], r["avg_ms"], r["avg_att"], r["n_launch"]
    achieved_ops, bytes_per_launch = r["achieved_ops"], r["bytes_per_launch"]
    profiled = (PROFILE is not None and PROFILE["kernel_src_sha256"] == kernel_src_sha256()
                and w["layout"] == "bitpack64")
    traffic = PROFILE["bytes_per_launch"] if profiled else None
    sweep_rate = avg_att / (avg_ms * 1e-3)
    hbm_GBs = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    line = {
        "metric": "spin-flip attempts/s",
        "value": attempts / wall,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w["name"], "L": w["L"], "R": w["R"], "eps": w["eps"],
                   "beta_max": w["beta_max"], "n_sweeps": w["n_sweeps"], "layout": w["layout"],
                   "couplings": "+-J p=1/2", "seed_config": 3},
        "roofline": {
            "bound": "alu",
            "kernel": f"k_sweep<{w['layout']}, L=10, +-J> (gather + 10 bit-sliced sweeps + energy)",
            "achieved": achieved_ops / 1e12,
            "peak": VALU_PEAK_OPS / 1e12,
            "unit": "Tops/s",
            "frac": achieved_ops / VALU_PEAK_OPS,
            "ops_per_attempt": OPS_PER_ATTEMPT,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)",
            "traffic_GBs": None if traffic is None else traffic / (avg_ms * 1e-3) / 1e9,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": avg_ms,
            "launches": n_launch,
            "attempts_per_launch": avg_att,
            "sweep_attempts_per_s": sweep_rate,
            # the kernel against the rate of its random numbers alone: Philox
            # draws with nothing else computed, measured on this device
            "philox_only_attempts_per_s": ceil["philox_draws_per_s"],
            "frac_of_philox_only": sweep_rate / ceil["philox_draws_per_s"],
            # executed VALU lane-instructions per attempt (rocprofv3 SQ_INSTS_VALU
            # per launch x 64 / attempts), for the source the counters were taken on
            "executed_valu_per_attempt": PROFILE["valu_per_attempt"] if profiled else None,
            "hbm_algorithmic_GBs": hbm_GBs,
            "hbm_frac": hbm_GBs / HBM_PEAK_GBS,
            "copy_GBs_measured": copy_GBs,
            "hbm_frac_of_copy": hbm_GBs / copy_GBs,
            # measured on this device just before the timed steps: the issue rate
            # of two-source operations (v_add_u32; XOR and v_bitop3 run as fast)
            # and of three-source ones (v_bfe_u32; extracts, v_add3, 24-bit mads)
            "measured_valu_peak": ceil["valu_lane_ops_per_s"] / 1e12,
            "measured_valu3_peak": ceil["valu3_lane_ops_per_s"] / 1e12,
            "frac_of_measured_valu_peak": achieved_ops / ceil["valu_lane_ops_per_s"],
            "frac_of_measured_valu3_peak": achieved_ops / ceil["valu3_lane_ops_per_s"],
        },
        "sweep_fraction_of_wall": sum(sweep_ms) * 1e-3 / wall,
        "outside_sweep_us_per_step": 1e6 * (wall - sum(sweep_ms) * 1e-3) / args.steps,
        "autotune": tune,
        "layout_autotune": ltune,
        "anneals_completed": len(anneals),
        "steps_per_anneal": anneals,
        "beta_at_end": stats[-1][0] if stats else None,
    }
    print("# one whole anneal", file=sys.stderr, flush=True)
    line["whole_anneal"] = whole_anneal(pam, J, w, seed0 + 2000)
    if args.gauss_steps > 0:
        print(f"# Gaussian couplings: {args.gauss_steps} steps", file=sys.stderr, flush=True)
        line["gauss16"] = gauss_bench(pam, args.gauss_steps, args.warmup, not args.no_autotune)
    if args.real_steps > 0:
        print(f"# real Gaussian couplings: {args.real_steps} steps", file=sys.stderr, flush=True)
        line["gauss_real"] = gauss_real_bench(pam, args.real_steps, args.warmup,
                                              not args.no_autotune)
    if not args.no_int8:
        print("# int8 layout: C1 and C2 whole runs", file=sys.stderr, flush=True)
        line["int8"] = {"C1": linear_run(pam, C1, 1, False), "C2": linear_run(pam, C2, 2, True)}
    if not args.no_batched:
        print("# batched: 256 instances, one graph per step; back-to-back sample", file=sys.stderr,
              flush=True)
        line["batched"] = batched_bench(pam)
    if args.serve_seconds > 0:
        print(f"# serving: Poisson arrivals for {args.serve_seconds:.0f} s", file=sys.stderr,
              flush=True)
        line["serving"] = serving_bench(args.serve_seconds, args.serve_max_active or None)
    if args.serve_load_seconds > 0 and args.serve_seconds > 0:
        # the same request mix at a rate where requests overlap (the configured
        # rate keeps about one resident at a time on this device)
        print(f"# serving under load: {args.serve_load_rate:g} requests/s for "
              f"{args.serve_load_seconds:.0f} s", file=sys.stderr, flush=True)
        line["serving_load"] = serving_bench(args.serve_load_seconds,
                                             args.serve_max_active or None,
                                             rate=args.serve_load_rate)
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w)
        if "gauss16" in line:
            line["gauss16"]["cpu_baseline"] = gauss_cpu_baseline(GAUSS_WORKLOAD)
        if "gauss_real" in line:
            line["gauss_real"]["cpu_baseline"] = gauss_real_cpu_baseline(REAL_WORKLOAD)
        if "int8" in line:
            line["int8"]["C1"]["cpu_baseline"] = int8_cpu_baseline(C1, 1, False, C1["n_temps"] - 1)
            line["int8"]["C2"]["cpu_baseline"] = int8_cpu_baseline(C2, 2, True, 2)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
