"""Serving loop for population-annealing runs on one GPU (continuous batching).

Each request is one PA run (Amey & Machta, arXiv:1711.02146, Sec. II loop) on
one +-J instance: L, R, a linear schedule of n_temps inverse temperatures on
[0, beta_max] and n_sweeps sweeps per temperature.  Requests are admitted in
arrival order while their device footprint (``pa_workspace_bytes``) fits the
HBM budget; admitted populations stay resident on the GPU until their last
temperature.  Every tick advances resident populations by one temperature step
each in one ``pa_stepper_step`` call, so requests that arrive while others run
join the next tick and their work shares the same launches.

Which residents a tick includes is work-fair (virtual-time fair queueing with
a batching window): every resident carries the work it has received so far
(its step cost N_S L^3 R, plus a fixed charge for the per-step overhead, per
step taken); a tick includes every resident within `window` attempts of the
least-served one, and a newcomer starts level with the least-served resident.
A cheap run therefore steps on most ticks while an expensive one waits until
the others have received comparable work, so a small request is not held to
the pace of the largest one in the mix and a large one is not starved by a
stream of small ones.

Each population draws only its own Philox streams, so a request's results do
not depend on what else is resident: they equal the results of the same run
made alone.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    L: int
    R: int
    n_temps: int            # temperatures of the linear schedule, beta_0 = 0 included
    n_sweeps: int
    beta_max: float
    J: object               # couplings, 3 L^3 values of +-1 (numpy int8)
    seed: int               # population seed
    layout: str = "bitpack64"

    def schedule(self):
        # beta_k = beta_max k / (n_temps - 1), each computed directly
        return [self.beta_max * k / (self.n_temps - 1) for k in range(self.n_temps)]

    def attempts(self) -> int:
        """Spin-flip attempts of the whole run at the target size R."""
        return (self.n_temps - 1) * self.n_sweeps * self.L ** 3 * self.R

    def step_cost(self) -> int:
        """Spin-flip attempts of one temperature step at the target size R."""
        return self.n_sweeps * self.L ** 3 * self.R


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    footprint: int
    status: int = 0                     # 0, or the PA status that stopped the run
    final: dict = field(default_factory=dict)
    trajectory: list = field(default_factory=list)   # per-step observables (if kept)
    attempts: int = 0                   # sum over steps of n_sweeps N R~

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


# statuses of requests that never ran (the C ABI's codes)
STATUS_INVALID = -1     # PA_EINVAL: L above the library's maximum, or no step in the schedule
STATUS_TOO_LARGE = -2   # PA_ENOMEM: footprint above the whole HBM budget


class Scheduler:
    """Host-side admission: FIFO by arrival, admitted while the device footprint fits.

    ``footprint(request) -> bytes``.  A request larger than the whole budget is
    rejected at arrival (it could never be admitted).  Head-of-line order is kept:
    a later request never overtakes an earlier one that does not fit yet.
    """

    def __init__(self, hbm_budget: int, max_active: int, footprint):
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.footprint = footprint
        self.queue: deque = deque()
        self.in_use = 0
        self.active = 0
        self.rejected: list = []

    def arrive(self, req: Request):
        if self.footprint(req) > self.budget:
            self.rejected.append(req)
        else:
            self.queue.append(req)

    def admit(self):
        """Requests to start now, in arrival order."""
        out = []
        while self.queue and self.active < self.max_active:
            f = self.footprint(self.queue[0])
            if self.in_use + f > self.budget:
                break
            req = self.queue.popleft()
            self.in_use += f
            self.active += 1
            out.append(req)
        return out

    def release(self, req: Request):
        self.in_use -= self.footprint(req)
        self.active -= 1


class GpuBackend:
    """Resident populations on one GPU, stepped together by a Stepper."""

    def __init__(self, max_active: int, max_L: int, device=None):
        import torch

        import paper_1711_02146_amd as pam

        self.pam = pam
        pam.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self.stream = torch.cuda.Stream(device=self.device)
        self.stepper = pam.Stepper(max_active, max_L, self.stream, device=self.device)
        self.max_L = max_L
        self._fp_cache = {}

    def footprint(self, req: Request) -> int:
        key = (req.L, req.R, req.layout)
        if key not in self._fp_cache:
            p = self.pam.pa_params(L=req.L, R=req.R, capacity=0,
                                   layout=self.pam.LAYOUTS[req.layout], seed=0, flags=0,
                                   model=0)
            self._fp_cache[key] = self.pam.pa_workspace_bytes(p)
        return self._fp_cache[key]

    def create(self, req: Request):
        return self.pam.Population(req.L, req.R, req.J, req.seed, layout=req.layout,
                                   device=self.device, stream=self.stream)

    def step(self, pops, beta_next, n_sweeps):
        return self.stepper.step(pops, beta_next, n_sweeps)

    def free(self, pop):
        pop.close()

    def close(self):
        self.stepper.close()


class Server:
    """The request loop: admission, one step of every resident run per tick, retirement.

    ``backend`` provides footprint(req), create(req), step(pops, beta_next,
    n_sweeps) -> (observables, statuses), free(pop) and max_L; by default the
    GPU backend above.
    """

    def __init__(self, hbm_budget: int = 64 << 30, max_active: int = 256, max_L: int = 16,
                 keep_trajectory: bool = False, backend=None, device=None, fair: bool = True,
                 window: float = 2e9, step_overhead: float = 1e8):
        """fair: work-fair tick membership (else every resident steps every tick);
        window: attempts of lead over the least-served resident that still join a
        tick; step_overhead: attempts charged per step for the fixed per-step cost
        (about 0.1 ms of sweeping on MI355X)."""
        self.backend = backend if backend is not None else GpuBackend(max_active, max_L, device)
        self.fair = fair
        self.window = float(window)
        self.step_overhead = float(step_overhead)
        self.max_L = self.backend.max_L
        self.keep_trajectory = keep_trajectory
        self.sched = Scheduler(hbm_budget, max_active, self.backend.footprint)
        self.ticks = 0
        self.tick_sizes = []

    def run(self, requests, realtime: bool = True, tick_dt: float = 0.0, progress=None):
        """Serve ``requests`` (any order); returns the Results in request-id order.

        realtime: arrivals follow the wall clock (sleeping while idle).  With
        realtime=False, time is virtual: each tick advances it by tick_dt, so
        admission order and the mix of resident requests are reproducible.
        """
        be = self.backend
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        active = []   # [request, population, schedule, k, result, work received]
        results = {}
        t0 = time.perf_counter()
        vnow = 0.0

        def now():
            return time.perf_counter() - t0 if realtime else vnow

        while pending or self.sched.queue or active:
            t = now()
            while pending and pending[0].arrival <= t:
                self.sched.arrive(pending.popleft())
            for req in self.sched.rejected:
                results[req.rid] = Result(req.rid, req.arrival, t, t, be.footprint(req),
                                          status=STATUS_TOO_LARGE)
            self.sched.rejected.clear()
            for req in self.sched.admit():
                if req.L > self.max_L or req.n_temps < 2:
                    self.sched.release(req)
                    results[req.rid] = Result(req.rid, req.arrival, t, t, be.footprint(req),
                                              status=STATUS_INVALID)
                    continue
                res = Result(req.rid, req.arrival, t, t, be.footprint(req))
                start = min((a[5] for a in active), default=0.0)
                active.append([req, be.create(req), req.schedule(), 0, res, start])
            if not active:
                if pending:
                    if realtime:
                        time.sleep(max(0.0, pending[0].arrival - now()))
                    else:
                        vnow = max(vnow, pending[0].arrival)
                continue
            if self.fair:
                least = min(a[5] for a in active)
                chosen = [a for a in active if a[5] <= least + self.window]
            else:
                chosen = active
            for a in chosen:
                a[5] += a[0].step_cost() + self.step_overhead
            pops = [a[1] for a in chosen]
            beta_next = [a[2][a[3] + 1] for a in chosen]
            n_sweeps = [a[0].n_sweeps for a in chosen]
            obs, status = be.step(pops, beta_next, n_sweeps)
            del pops
            self.ticks += 1
            self.tick_sizes.append(len(chosen))
            if not realtime:
                vnow += tick_dt
            t = now()
            done = set()
            for a, o, st in zip(chosen, obs, status):
                req, _, sched, k, res = a[:5]
                if st != 0:
                    res.status = int(st)
                    res.finished = t
                    self._retire(a, results)
                    done.add(id(a))
                    continue
                a[3] = k + 1
                res.attempts += req.n_sweeps * req.L ** 3 * o["R_tilde"]
                if self.keep_trajectory:
                    res.trajectory.append(o)
                if a[3] == len(sched) - 1:
                    res.final = o
                    res.finished = t
                    self._retire(a, results)
                    done.add(id(a))
            active = [a for a in active if id(a) not in done]
            if progress is not None:
                progress(t, len(results), len(active), len(self.sched.queue))
        return [results[k] for k in sorted(results)]

    def _retire(self, a, results):
        req, pop, _, _, res = a[:5]
        self.backend.free(pop)
        a[1] = None
        self.sched.release(req)
        results[req.rid] = res

    def close(self):
        if hasattr(self.backend, "close"):
            self.backend.close()
