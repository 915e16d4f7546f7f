"""Scheduling logic of the continuous-batching service, driven by a host-side
engine with a simulated clock (no GPU)."""
import numpy as np
import pytest

from paper_1712_05012_amd.serve import FoldService, Job


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class HostEngine:
    """Each job converges after `conv[job_id]` iterations (or never if None);
    a job listed in `fail` reports a numeric failure on its first tick."""

    def __init__(self, clock, conv, fail=(), bytes_per_atom=1000, tick_seconds=0.01, chain_seconds=0.0):
        self.clock, self.conv, self.fail = clock, conv, set(fail)
        self.bpa, self.dt, self.dc = bytes_per_atom, tick_seconds, chain_seconds
        self.open_bytes = 0
        self.peak_bytes = 0
        self.events = []

    def bytes_for(self, job):
        return self.bpa * job.n_atoms

    def open(self, job):
        self.open_bytes += self.bytes_for(job)
        self.peak_bytes = max(self.peak_bytes, self.open_bytes)
        self.events.append(("open", job.job_id, self.clock()))
        return {"job": job, "iters": 0}

    def step(self, chains, n_iter):
        self.clock.t += self.dt + self.dc * len(chains)
        out = []
        for c in chains:
            j = c["job"]
            if j.job_id in self.fail:
                out.append((c["iters"], False, -4))
                continue
            target = self.conv.get(j.job_id)
            lim = j.max_iter if target is None else min(target, j.max_iter)
            c["iters"] = min(c["iters"] + n_iter, lim)
            out.append((c["iters"], target is not None and c["iters"] >= target, 0))
        return out

    def theta(self, chain):
        return np.zeros(2 * len(chain["job"].res_type))

    def close(self, chain):
        self.open_bytes -= self.bytes_for(chain["job"])
        self.events.append(("close", chain["job"].job_id, self.clock()))


def make_jobs(n, lengths, arrivals, max_iter=200):
    return [Job(job_id=k, res_type=np.zeros(lengths[k], np.int32), theta0=np.zeros(2 * lengths[k]),
                arrival=arrivals[k], max_iter=max_iter) for k in range(n)]


def test_budget_never_exceeded_and_every_job_finishes():
    clk = SimClock()
    rng = np.random.default_rng(0)
    n = 40
    lengths = rng.integers(30, 300, n)
    arrivals = np.cumsum(rng.exponential(0.02, n))
    conv = {k: int(rng.integers(20, 150)) for k in range(n) if k % 3}
    eng = HostEngine(clk, conv)
    budget = 1000 * 10 * 700  # room for a few chains at a time
    svc = FoldService(eng, hbm_budget=budget, max_slots=8, check_every=10, clock=clk, sleep=clk.sleep)
    st = svc.run(make_jobs(n, lengths, arrivals))
    assert len(st.jobs) == n
    assert eng.peak_bytes <= budget
    assert st.max_live <= 8
    for j in st.jobs:
        assert j.finished >= j.admitted >= j.arrival
        if j.job_id in conv:
            assert j.converged and j.iterations == conv[j.job_id]
        else:
            assert not j.converged and j.iterations == j.max_iter
    s = st.summary()
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0
    assert st.atom_steps == sum(j.n_atoms * j.iterations for j in st.jobs)


def test_admission_in_arrival_order_and_refill_mid_flight():
    clk = SimClock()
    lengths = [100] * 6
    arrivals = [0.0, 0.0, 0.005, 0.006, 0.5, 0.5]
    conv = {0: 30, 1: 200, 2: 30, 3: 30, 4: 30, 5: 30}
    eng = HostEngine(clk, conv)
    svc = FoldService(eng, hbm_budget=10**9, max_slots=2, check_every=10, clock=clk, sleep=clk.sleep)
    st = svc.run(make_jobs(6, lengths, arrivals, max_iter=500))
    opens = [e[1] for e in eng.events if e[0] == "open"]
    assert opens == sorted(opens)
    # job 2 (arrived while 0 and 1 were live) starts only when job 0 frees its slot
    close0 = [e[2] for e in eng.events if e == ("close", 0, e[2])][0]
    open2 = [e[2] for e in eng.events if e[0] == "open" and e[1] == 2][0]
    assert open2 >= close0
    # and it runs while job 1 is still on the device
    close1 = [e[2] for e in eng.events if e[0] == "close" and e[1] == 1][0]
    assert open2 < close1
    assert st.queue_peak >= 1


def test_failed_job_is_retired_without_disturbing_others():
    clk = SimClock()
    eng = HostEngine(clk, {0: 40, 2: 40}, fail={1})
    svc = FoldService(eng, hbm_budget=10**9, max_slots=4, check_every=10, clock=clk, sleep=clk.sleep)
    st = svc.run(make_jobs(3, [50, 50, 50], [0.0, 0.0, 0.0]))
    by = {j.job_id: j for j in st.jobs}
    assert by[1].status == -4 and not by[1].converged
    assert by[0].converged and by[2].converged
    assert st.summary()["failed"] == 1


def test_job_larger_than_budget_is_refused():
    clk = SimClock()
    eng = HostEngine(clk, {})
    svc = FoldService(eng, hbm_budget=1000, max_slots=4, clock=clk, sleep=clk.sleep)
    with pytest.raises(ValueError):
        svc.run(make_jobs(1, [50], [0.0]))


def _stream(n, gap, max_iter):
    return make_jobs(n, [50] * n, [k * gap for k in range(n)], max_iter=max_iter)


def test_queue_growth_reports_overload_and_not_underload():
    # each job needs 5 ticks (50 iterations / 10 per tick) of 0.01 s on one slot
    clk = SimClock()
    over = FoldService(HostEngine(clk, {}), hbm_budget=10**9, max_slots=1, check_every=10,
                       clock=clk, sleep=clk.sleep)
    st = over.run(_stream(60, 0.01, 50))        # 100 jobs/s offered, 20 jobs/s served
    s = st.summary(skip=10)
    assert s["jobs"] == 50 and s["warmup_jobs_discarded"] == 10
    # the waiting queue grows by about 100 - 20 = 80 jobs/s while jobs arrive
    assert 60.0 < s["queue_growth_jobs_per_s"] < 100.0
    assert s["queue_at_last_arrival"] > 30
    assert s["backlog_growth_jobs_per_s"] >= s["queue_growth_jobs_per_s"] - 1e-9


def test_backlog_growth_sees_jobs_held_in_slots():
    # enough slots to admit everything: the queue stays short while the live
    # set grows by the excess of arrivals over completions.  A tick costs
    # 0.01 s + 1 ms per live chain and a job needs 5 ticks, so at most
    # 1 / (5 * 1 ms) = 200 jobs/s complete while 500 jobs/s arrive.
    clk = SimClock()
    svc = FoldService(HostEngine(clk, {}, chain_seconds=1e-3), hbm_budget=10**9, max_slots=10000,
                      check_every=10, clock=clk, sleep=clk.sleep)
    st = svc.run(_stream(400, 0.002, 50))
    s = st.summary()
    assert s["backlog_growth_jobs_per_s"] > 200.0
    assert s["queue_growth_jobs_per_s"] < s["backlog_growth_jobs_per_s"] / 4
    assert s["served_jobs_per_s"] < 200.0

    clk = SimClock()
    under = FoldService(HostEngine(clk, {}), hbm_budget=10**9, max_slots=8, check_every=10,
                        clock=clk, sleep=clk.sleep)
    st = under.run(_stream(60, 0.02, 50))       # 50 jobs/s offered, up to 160 jobs/s served
    s = st.summary(skip=10)
    assert abs(s["queue_growth_jobs_per_s"]) < 5.0
    assert s["queue_at_last_arrival"] <= 1
    assert abs(s["backlog_growth_jobs_per_s"]) < 5.0
    # latency is the service time alone: 5 ticks
    assert s["p99_latency_s"] == pytest.approx(0.05, abs=0.011)


def test_warmup_discard_drops_the_earliest_arrivals():
    clk = SimClock()
    svc = FoldService(HostEngine(clk, {}), hbm_budget=10**9, max_slots=1, check_every=10,
                      clock=clk, sleep=clk.sleep)
    st = svc.run(_stream(20, 0.001, 20))
    all_lat = sorted(j.latency for j in st.jobs)
    kept = sorted(j.latency for j in st.jobs if j.job_id >= 5)
    s = st.summary(skip=5)
    assert s["jobs"] == 15
    assert s["p50_latency_s"] == pytest.approx(float(np.percentile(kept, 50)))
    assert s["p50_latency_s"] > float(np.percentile(all_lat[:5], 50))
