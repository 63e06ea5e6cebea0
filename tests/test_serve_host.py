"""Host logic of the serving loop (CPU): admission by device footprint, the
request loop's bookkeeping with a stand-in backend, and the request stream."""
import math

import numpy as np

import pa_inputs
from paper_1711_02146_amd.serve import (STATUS_INVALID, STATUS_TOO_LARGE, Request, Scheduler,
                                        Server)


def req(rid, arrival, R, L=4, n_temps=5):
    return Request(rid=rid, arrival=arrival, L=L, R=R, n_temps=n_temps, n_sweeps=10, beta_max=5.0,
                   J=None, seed=rid)


def test_scheduler_fifo_budget_and_rejection():
    s = Scheduler(hbm_budget=100, max_active=10, footprint=lambda r: r.R)
    for r in [req(0, 0, 60), req(1, 0, 50), req(2, 0, 30), req(3, 0, 101)]:
        s.arrive(r)
    assert [r.rid for r in s.rejected] == [3]           # larger than the whole budget
    assert [r.rid for r in s.admit()] == [0]            # 1 does not fit; 2 must not overtake it
    assert s.in_use == 60 and [r.rid for r in s.queue] == [1, 2]
    s.release(req(0, 0, 60))
    assert [r.rid for r in s.admit()] == [1, 2]
    assert s.in_use == 80 and s.active == 2


def test_scheduler_max_active():
    s = Scheduler(hbm_budget=10 ** 9, max_active=2, footprint=lambda r: 1)
    for i in range(5):
        s.arrive(req(i, 0, 1))
    assert len(s.admit()) == 2 and len(s.admit()) == 0
    s.release(req(0, 0, 1))
    assert [r.rid for r in s.admit()] == [2]


class FakeBackend:
    """Stands in for the GPU: records what the loop asks of it."""
    max_L = 16

    def __init__(self, budget):
        self.budget = budget
        self.resident = {}
        self.max_in_use = 0
        self.calls = []
        self.fail_at = {}   # rid -> step index that reports a capacity overflow

    def footprint(self, r):
        return r.R

    def create(self, r):
        h = {"req": r, "k": 0}
        self.resident[r.rid] = h
        self.max_in_use = max(self.max_in_use, sum(x["req"].R for x in self.resident.values()))
        return h

    def step(self, pops, beta_next, n_sweeps):
        self.calls.append([p["req"].rid for p in pops])
        obs, st = [], []
        for p, b, n in zip(pops, beta_next, n_sweeps):
            r = p["req"]
            assert b == r.schedule()[p["k"] + 1] and n == r.n_sweeps
            if self.fail_at.get(r.rid) == p["k"]:
                obs.append({})
                st.append(-3)
                continue
            p["k"] += 1
            obs.append({"R_tilde": r.R, "beta": b, "k": p["k"]})
            st.append(0)
        return obs, np.array(st, np.int32)

    def free(self, p):
        del self.resident[p["req"].rid]


def test_server_loop_virtual_time():
    be = FakeBackend(budget=250)
    srv = Server(hbm_budget=250, max_active=8, backend=be, keep_trajectory=True)
    reqs = [req(0, 0.0, 100, n_temps=6), req(1, 0.01, 100, n_temps=3), req(2, 0.02, 100),
            req(3, 0.5, 300), req(4, 0.07, 40, L=18), req(5, 0.08, 40, n_temps=1),
            req(6, 0.2, 50, n_temps=4)]
    be.fail_at[6] = 1
    res = srv.run(reqs, realtime=False, tick_dt=0.01)
    by = {r.rid: r for r in res}
    assert sorted(by) == list(range(7))
    assert by[3].status == STATUS_TOO_LARGE
    assert by[4].status == STATUS_INVALID and by[5].status == STATUS_INVALID
    assert by[6].status == -3 and len(by[6].trajectory) == 1
    for i in (0, 1, 2):
        r = by[i]
        assert r.status == 0
        assert len(r.trajectory) == reqs[i].n_temps - 1
        assert [o["k"] for o in r.trajectory] == list(range(1, reqs[i].n_temps))
        assert r.final["beta"] == 5.0
        assert r.attempts == (reqs[i].n_temps - 1) * 10 * 64 * reqs[i].R
        assert r.finished >= r.admitted >= r.arrival
    # the budget held: 0 and 1 ran together, 2 waited for 1 to leave
    assert be.max_in_use <= 250
    assert by[2].admitted >= by[1].finished
    assert not be.resident and srv.sched.in_use == 0 and srv.sched.active == 0
    # requests joined running work: some tick stepped two requests at once
    assert max(len(c) for c in be.calls) >= 2
    assert sum(len(c) for c in be.calls) == 5 + 2 + 4 + 2


def test_serving_request_stream():
    rs = pa_inputs.serving_requests(duration_s=600.0, rate=4.0)
    n = len(rs)
    # Poisson count over 600 s at 4/s: 2400 +- 49
    assert abs(n - 2400) < 5 * math.sqrt(2400)
    t = np.array([r["arrival"] for r in rs])
    assert np.all(np.diff(t) > 0) and t[-1] <= 600.0
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.25) < 5 * 0.25 / math.sqrt(n)
    assert {r["L"] for r in rs} == {4, 6, 8, 10, 12}
    R = np.array([r["R"] for r in rs], float)
    assert R.min() >= 1e4 and R.max() <= 2e5
    # log-uniform: ln R uniform on [ln 1e4, ln 2e5]
    u = (np.log(R) - np.log(1e4)) / (np.log(2e5) - np.log(1e4))
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / n)
    nt = np.array([r["n_temps"] for r in rs])
    assert nt.min() >= 51 and nt.max() <= 201
    # the same seed gives the same stream
    assert pa_inputs.serving_requests(duration_s=10.0) == pa_inputs.serving_requests(duration_s=10.0)


def test_server_work_fair_ticks():
    """Fair queueing by work received: a run whose steps cost 4x another's joins a
    tick only once the cheap run has caught up; both finish all steps in order."""
    be = FakeBackend(budget=10 ** 9)
    srv = Server(hbm_budget=10 ** 9, max_active=8, backend=be, keep_trajectory=True,
                 window=0.0, step_overhead=0.0)
    cheap = req(0, 0.0, 100, n_temps=13)      # step cost 10 * 64 * 100
    dear = req(1, 0.0, 400, n_temps=4)        # 4x that
    res = srv.run([cheap, dear], realtime=False, tick_dt=0.01)
    assert [r.status for r in res] == [0, 0]
    assert len(res[0].trajectory) == 12 and len(res[1].trajectory) == 3
    assert all(0 in c for c in be.calls[:12])
    assert [i for i, c in enumerate(be.calls) if 1 in c] == [0, 4, 8]
    # a window wider than the whole run lets both step on every tick
    be1 = FakeBackend(budget=10 ** 9)
    Server(hbm_budget=10 ** 9, max_active=8, backend=be1, window=1e12,
           step_overhead=0.0).run([cheap, dear], realtime=False, tick_dt=0.01)
    assert [sorted(c) for c in be1.calls[:3]] == [[0, 1]] * 3
    # without fairness every resident steps on every tick
    be2 = FakeBackend(budget=10 ** 9)
    Server(hbm_budget=10 ** 9, max_active=8, backend=be2, fair=False).run(
        [cheap, dear], realtime=False, tick_dt=0.01)
    assert [sorted(c) for c in be2.calls[:3]] == [[0, 1]] * 3
    # a newcomer starts level with the least-served resident
    be3 = FakeBackend(budget=10 ** 9)
    late = req(2, 0.05, 100, n_temps=3)
    srv3 = Server(hbm_budget=10 ** 9, max_active=8, backend=be3, window=0.0, step_overhead=0.0)
    srv3.run([cheap, dear, late], realtime=False, tick_dt=0.01)
    first_late = next(i for i, c in enumerate(be3.calls) if 2 in c)
    assert first_late == 5 and 0 in be3.calls[first_late]
