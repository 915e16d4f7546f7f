"""Continuous-batching folding service on one GPU.

Jobs (a sequence, a start conformation, a tolerance and an iteration cap)
arrive over time.  The scheduler admits a waiting job as soon as a slot and
enough of the HBM budget are free, builds its chain on the device, and every
tick advances all live chains together with one ``kcm_step`` call of
``check_every`` iterations.  After each tick it reads the per-chain reports,
retires every chain that converged (max|dtheta| < tol), reached its
iteration cap, or failed numerically, frees its memory, and admits the next
waiting jobs, so new work overlaps with work already on the device.

The device engine is ``KcmEngine`` (the C ABI through the binding); the
scheduler only sees its small interface, so its bookkeeping can also be
driven by a host-side engine in tests.
"""
from __future__ import annotations

import heapq
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Job:
    job_id: int
    res_type: np.ndarray
    theta0: np.ndarray
    arrival: float                 # seconds on the service clock
    tol: float = 1e-4              # convergence threshold on max|dtheta| (rad)
    max_iter: int = 2000
    # filled in by the service
    admitted: float = float("nan")
    finished: float = float("nan")
    iterations: int = 0
    converged: bool = False
    status: int = 0
    theta: np.ndarray | None = None
    bytes: int = 0

    @property
    def n_atoms(self) -> int:
        return 10 * int(len(self.res_type))

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class KcmEngine:
    """Device engine: chains in torch-allocated blocks, stepped through libkcm."""

    def __init__(self, residue_types, params=None, stream=None):
        from . import kcm

        self.kcm = kcm
        self.types = residue_types
        self.params = params if params is not None else kcm.kcm_default_params(precision=kcm.KCM_MIXED)
        self.stream = stream

    def bytes_for(self, job: Job) -> int:
        return self.kcm.kcm_chain_bytes(self.kcm.make_desc(job.res_type, self.types), self.params) + 256

    def open(self, job: Job):
        chain = self.kcm.Chain(job.res_type, self.types, self.params, theta0=job.theta0, stream=self.stream)
        self.kcm.kcm_set_limits(chain.handle, job.tol, job.max_iter, self.stream)
        return chain

    def step(self, chains, n_iter: int):
        """Advance every chain by up to n_iter iterations: [(iterations, converged, status)]."""
        _, reps = self.kcm.kcm_step(chains, n_iter, self.stream, report=True, check=False)
        return [(int(r.iterations), bool(r.converged), int(r.status)) for r in reps]

    def theta(self, chain):
        return chain.theta(self.stream)

    def close(self, chain):
        chain.free()


@dataclass
class ServiceStats:
    jobs: list = field(default_factory=list)
    atom_steps: int = 0
    wall: float = 0.0
    ticks: int = 0
    max_live: int = 0
    max_bytes: int = 0
    queue_peak: int = 0
    queue_trace: list = field(default_factory=list)  # (service time, waiting, live) before each tick
    last_arrival: float = 0.0

    def growth(self, t_from: float = 0.0, live: bool = False):
        """Least-squares slope (jobs/s) of the waiting queue (``live``: of the
        jobs in the system, waiting plus live) while jobs still arrive.

        Ticks from ``t_from`` up to the last arrival count; a slope well above
        zero means the offered load exceeds what the device serves."""
        pts = [(t, q + (n if live else 0)) for t, q, n in self.queue_trace if t_from <= t <= self.last_arrival]
        if len(pts) < 2:
            return None
        t = np.array([p[0] for p in pts])
        q = np.array([p[1] for p in pts], dtype=np.float64)
        if np.ptp(t) <= 0:
            return None
        return float(np.polyfit(t, q, 1)[0])

    def summary(self, skip: int = 0):
        """Latency over the jobs after the first ``skip`` (by job id, i.e. arrival order)."""
        done = [j for j in self.jobs[skip:]]
        lat = np.array([j.latency for j in done]) if done else np.zeros(0)
        t_warm = min((j.arrival for j in done), default=0.0)
        q_end = [q for t, q, _ in self.queue_trace if t <= self.last_arrival]
        return {
            "jobs": len(done),
            "warmup_jobs_discarded": int(min(skip, len(self.jobs))),
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_iterations": float(np.mean([j.iterations for j in done])) if done else None,
            "atom_steps_per_s": self.atom_steps / self.wall if self.wall > 0 else None,
            "wall_s": self.wall,
            "converged": int(sum(j.converged for j in done)),
            "failed": int(sum(j.status != 0 for j in done)),
            "failed_jobs": [{"job_id": j.job_id, "status": j.status, "iterations": j.iterations,
                             "residues": int(len(j.res_type))} for j in self.jobs if j.status != 0][:20],
            "status_counts": {str(k): int(v) for k, v in
                              zip(*np.unique([j.status for j in done], return_counts=True))} if done else {},
            "ticks": self.ticks,
            "max_live": self.max_live,
            "max_bytes": self.max_bytes,
            "queue_peak": self.queue_peak,
            "queue_at_last_arrival": int(q_end[-1]) if q_end else 0,
            "queue_growth_jobs_per_s": self.growth(t_warm),
            "backlog_growth_jobs_per_s": self.growth(t_warm, live=True),
            "served_jobs_per_s": len(self.jobs) / self.wall if self.wall > 0 else None,
        }


class FoldService:
    """Admission by HBM budget into at most ``max_slots`` live chains."""

    def __init__(self, engine, hbm_budget: int, max_slots: int = 1024, check_every: int = 10,
                 clock=time.perf_counter, sleep=time.sleep):
        if hbm_budget <= 0 or max_slots <= 0 or check_every <= 0:
            raise ValueError("hbm_budget, max_slots and check_every must be positive")
        self.engine = engine
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.check_every = int(check_every)
        self.clock = clock
        self.sleep = sleep

    def run(self, jobs, on_retire=None):
        """Serve ``jobs`` (arrival times relative to the start) to completion.

        ``on_retire(job, n_done)``, if given, is called as each job retires."""
        pending = sorted(jobs, key=lambda j: (j.arrival, j.job_id))
        for j in pending:
            j.bytes = self.engine.bytes_for(j)
            if j.bytes > self.budget:
                raise ValueError(f"job {j.job_id} needs {j.bytes} B, more than the whole budget")
        waiting: list = []                 # (arrival, job_id, job) min-heap
        live: dict = {}                    # job_id -> (job, chain, start_iterations)
        used = 0
        stats = ServiceStats()
        stats.last_arrival = max((j.arrival for j in pending), default=0.0)
        t0 = self.clock()
        nxt = 0
        while nxt < len(pending) or waiting or live:
            now = self.clock() - t0
            while nxt < len(pending) and pending[nxt].arrival <= now:
                j = pending[nxt]
                heapq.heappush(waiting, (j.arrival, j.job_id, j))
                nxt += 1
            stats.queue_peak = max(stats.queue_peak, len(waiting))
            # admit in arrival order while a slot and the memory are free
            while waiting and len(live) < self.max_slots and used + waiting[0][2].bytes <= self.budget:
                _, _, j = heapq.heappop(waiting)
                chain = self.engine.open(j)
                j.admitted = self.clock() - t0
                used += j.bytes
                live[j.job_id] = (j, chain, 0)
            stats.max_live = max(stats.max_live, len(live))
            stats.max_bytes = max(stats.max_bytes, used)
            if not live:
                if nxt < len(pending):
                    self.sleep(max(0.0, pending[nxt].arrival - (self.clock() - t0)))
                continue
            order = sorted(live)
            chains = [live[k][1] for k in order]
            stats.queue_trace.append((now, len(waiting), len(live)))
            reports = self.engine.step(chains, self.check_every)
            stats.ticks += 1
            now = self.clock() - t0
            for k, (iters, converged, status) in zip(order, reports):
                j, chain, _ = live[k]
                stats.atom_steps += j.n_atoms * (iters - j.iterations)
                j.iterations = iters
                if status != 0 or converged or iters >= j.max_iter:
                    j.status = int(status)
                    j.converged = bool(converged)
                    j.theta = self.engine.theta(chain)
                    j.finished = now
                    self.engine.close(chain)
                    used -= j.bytes
                    del live[k]
                    stats.jobs.append(j)
                    if on_retire is not None:
                        on_retire(j, len(stats.jobs))
        stats.wall = self.clock() - t0
        stats.jobs.sort(key=lambda j: j.job_id)
        return stats
