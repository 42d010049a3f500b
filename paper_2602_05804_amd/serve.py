"""Continuous-batching serving loop for independent gravity solves.

A request is one particle system (x, m, h; v = 0) to be evolved for a few
kick-drift-kick leapfrog steps (one solve per step plus the initial one).
Requests arrive over time; the loop

  * queues arrivals in FIFO order;
  * admits the head of the queue while its device footprint fits the HBM
    budget and a slot is free (a request larger than the whole budget fails
    at once instead of blocking the queue);
  * at every tick advances every admitted request by one step: the active
    systems are packed into forest solves of a bounded number of particles
    (``Solver.solve_batch``: one pass of every kernel for all systems of a
    pack);
  * frees a request's slot when its last step is done, so waiting requests
    join at the next tick (the set of systems in a packed solve changes from
    tick to tick);
  * isolates failures: a solve that raises fails only its own request(s),
    as long as the error leaves the device usable (bad input, unsupported
    configuration, out of memory); a HIP error (SFMM_EDEVICE) may leave the
    device in a faulted state, so it ends the run (``DeviceFault``) instead
    of being retried on the same device.

The executor is pluggable so that admission, ordering, slot release and
failure handling can be exercised without a GPU (``FakeExecutor``).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


class DeviceFault(RuntimeError):
    """A solve failed with a HIP error: the device may be unusable, so the
    serving loop stops (a caller may start a fresh process)."""


# sfmm_status codes after which the device is still usable: the failing
# systems are retried one by one and only they fail
RECOVERABLE = (-1, -2, -4, -5)  # EINVAL, ENOMEM, EUNSUPPORTED, ENONFINITE


def solve_packs(packs, solve_pack, solve_one, on_result, on_error):
    """Solve every pack with solve_pack(pack) -> results (one per system).
    If a pack fails with a recoverable status, its systems are solved one by
    one with solve_one(job) and only those that fail again get on_error(job,
    message).  Any other failure (a HIP error, or an error without a status
    code) raises DeviceFault at once."""
    for pack in packs:
        try:
            res = solve_pack(pack)
        except Exception as e:
            if getattr(e, "code", 0) not in RECOVERABLE:
                raise DeviceFault(f"packed solve failed: {e}") from e
            for j in pack:
                try:
                    on_result(j, solve_one(j))
                except Exception as e1:
                    if getattr(e1, "code", 0) not in RECOVERABLE:
                        raise DeviceFault(f"solve of request {j.rid} failed: {e1}") from e1
                    on_error(j, str(e1))
            continue
        for j, r in zip(pack, res):
            on_result(j, r)


@dataclass
class Job:
    rid: int
    arrival: float
    n: int
    steps: int
    dt: float
    payload: object = None          # host arrays (x, m, h) until admitted
    state: dict = field(default_factory=dict)  # device buffers while active
    step_done: int = -1             # -1: initial solve pending
    admitted_at: float = math.nan
    finished_at: float = math.nan
    error: Optional[str] = None

    @property
    def done(self) -> bool:
        return self.step_done >= self.steps


class FakeExecutor:
    """CPU stand-in: a step costs `sec_per_particle` * sum of N; footprint is
    `bytes_per_particle` * N.  `fail_rid` makes the solves of one request raise."""

    def __init__(self, sec_per_particle=1e-8, bytes_per_particle=1000, fail_rid=None):
        self.sec_per_particle = sec_per_particle
        self.bytes_per_particle = bytes_per_particle
        self.fail_rid = fail_rid
        self.ticks: List[List[int]] = []

    def footprint(self, n: int) -> int:
        return self.bytes_per_particle * n

    def admit(self, job: Job):
        job.state = {"n": job.n}

    def release(self, job: Job):
        job.state = {}

    def step(self, jobs: List[Job]):
        self.ticks.append([j.rid for j in jobs])
        time.sleep(self.sec_per_particle * sum(j.n for j in jobs))
        for j in jobs:
            if self.fail_rid is not None and j.rid == self.fail_rid:
                j.error = "injected failure"
            else:
                j.step_done += 1


class GpuExecutor:
    """Runs steps on the GPU through libsfmm.  At every tick the active
    systems are grouped, in admission order, into packs of at most
    `pack_particles` particles, and each pack is one packed solve
    (``Solver.solve_batch``): one pass of every kernel for all of its systems.
    A system larger than the cap is a pack of its own.  When a packed solve
    fails, its systems are solved one by one so that only the failing
    requests fail.  `tuned` maps size buckets (powers of two) to Solver
    arguments (autotune.tune_buckets): each pack is solved with those of the
    bucket nearest to its particle count, one Solver per distinct setting."""

    def __init__(self, precision="fp64", theta=0.5, order=3, pack_particles=16_000_000,
                 bytes_per_particle=None, tuned=None, **solver_cfg):
        import torch

        import paper_2602_05804_amd as sfmm

        self.torch = torch
        self.sfmm = sfmm
        self.precision = precision
        self.theta = theta
        self.order = order
        self.pack_particles = int(pack_particles)
        self.solver_cfg = solver_cfg
        self.tuned = dict(tuned or {})
        self.solver = sfmm.Solver(**solver_cfg)
        self._solvers = {(): self.solver}
        self.stream = torch.cuda.Stream()
        # per-particle device bytes: the context's workspace plus the request's
        # own buffers (x, v, m, h, acc, pot); measured once if not given
        self.bytes_per_particle = bytes_per_particle or self._measure_bytes()

    def _measure_bytes(self, n=20000):
        torch = self.torch
        g = torch.Generator(device="cuda").manual_seed(0)
        x = torch.rand((n, 3), dtype=torch.float64, device="cuda", generator=g)
        m = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
        h = torch.full((n,), 0.05, dtype=torch.float64, device="cuda")
        s = self.sfmm.Solver(**self.solver_cfg)
        s.solve(x, m, h, theta=self.theta, order=self.order, precision=self.precision)
        torch.cuda.synchronize()
        b = s.workspace_bytes() / n
        s.close()
        return int(b * 1.5) + 12 * 8  # slack for list growth + request buffers

    def solver_for(self, n: int):
        """The Solver for a pack of n particles (tuned, else the default)."""
        from paper_2602_05804_amd import autotune

        cfg = autotune.config_for(self.tuned, n)
        key = tuple(sorted(cfg.items()))
        if key not in self._solvers:
            self._solvers[key] = self.sfmm.Solver(**{**self.solver_cfg, **cfg})
        return self._solvers[key]

    def footprint(self, n: int) -> int:
        return self.bytes_per_particle * n

    def admit(self, job: Job):
        torch = self.torch
        x, m, h = job.payload
        dev = torch.device("cuda")
        st = {"x": torch.from_numpy(np.ascontiguousarray(x)).to(dev),
              "m": torch.from_numpy(np.ascontiguousarray(m)).to(dev),
              "h": torch.from_numpy(np.ascontiguousarray(h)).to(dev)}
        st["v"] = torch.zeros_like(st["x"])
        st["acc"] = torch.empty_like(st["x"])
        torch.cuda.current_stream().synchronize()  # the steps run on another stream
        job.state = st
        job.payload = None

    def release(self, job: Job):
        job.state = {}

    def _advance(self, job: Job, acc):
        """Leapfrog bookkeeping after the solve that produced `acc`."""
        st = job.state
        st["acc"] = acc
        k = job.step_done + 1  # index of the solve just done (0 = initial)
        if k == job.steps:
            self.sfmm.leapfrog(st["x"], st["v"], acc, 0.5 * job.dt, 0.0)  # closing half kick
        job.step_done = k

    def _pre(self, job: Job):
        """Kick + drift before the next solve."""
        k = job.step_done + 1
        if k >= 1:
            kick = 0.5 * job.dt if k == 1 else job.dt
            self.sfmm.leapfrog(job.state["x"], job.state["v"], job.state["acc"], kick, job.dt)

    def packs(self, jobs: List[Job]) -> List[List[Job]]:
        out, cur, n = [], [], 0
        for j in jobs:
            if cur and n + j.n > self.pack_particles:
                out.append(cur)
                cur, n = [], 0
            cur.append(j)
            n += j.n
        if cur:
            out.append(cur)
        return out

    def step(self, jobs: List[Job]):
        torch = self.torch
        packs = self.packs(jobs)

        def solve_pack(pack):
            for j in pack:
                self._pre(j)
            solver = self.solver_for(sum(j.n for j in pack))
            res = solver.solve_batch(
                [(j.state["x"], j.state["m"], j.state["h"]) for j in pack],
                theta=self.theta, order=self.order, precision=self.precision)
            return [a.clone() for a, _ in res]

        def solve_one(j):
            a, _ = self.solver_for(j.n).solve(j.state["x"], j.state["m"], j.state["h"],
                                              theta=self.theta, order=self.order,
                                              precision=self.precision)
            return a

        def on_error(j, msg):
            j.error = msg

        with torch.cuda.stream(self.stream):
            solve_packs(packs, solve_pack, solve_one, self._advance, on_error)
        self.stream.synchronize()


@dataclass
class Report:
    completed: int
    failed: int
    rejected: int
    makespan_s: float
    latencies_s: List[float]
    solves: int
    particle_solves: int
    max_active: int
    ticks: int
    tick_s: List[float] = field(default_factory=list)

    def summary(self) -> dict:
        lat = np.array(self.latencies_s) if self.latencies_s else np.array([math.nan])
        tk = np.array(self.tick_s) if self.tick_s else np.array([math.nan])
        return {"completed": self.completed, "failed": self.failed, "rejected": self.rejected,
                "makespan_s": self.makespan_s,
                "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
                "solves_per_s": self.solves / self.makespan_s if self.makespan_s > 0 else 0.0,
                "particles_per_s": (self.particle_solves / self.makespan_s
                                    if self.makespan_s > 0 else 0.0),
                "p50_step_ms": float(np.percentile(tk, 50) * 1e3),
                "p99_step_ms": float(np.percentile(tk, 99) * 1e3),
                "max_active": self.max_active, "ticks": self.ticks}


class Server:
    def __init__(self, executor, hbm_budget: float, max_active: int = 1024,
                 max_particles: float = math.inf,
                 clock: Callable[[], float] = time.perf_counter):
        """hbm_budget: bytes of device memory for admitted requests;
        max_particles: particles in flight (bounds the time of one step)."""
        self.ex = executor
        self.budget = float(hbm_budget)
        self.max_active = max_active
        self.max_particles = float(max_particles)
        self.clock = clock

    def run(self, jobs: List[Job], realtime: bool = True) -> Report:
        """Serve `jobs`.  With realtime, arrival times are seconds after the
        start of the run; without, every job is queued at once."""
        pending = sorted(jobs, key=lambda j: j.arrival)
        queue: List[Job] = []
        active: List[Job] = []
        done: List[Job] = []
        used = 0.0
        inflight = 0
        t0 = self.clock()
        solves = psolves = ticks = max_act = rejected = 0
        tick_s: List[float] = []
        while pending or queue or active:
            now = self.clock() - t0 if realtime else math.inf
            while pending and pending[0].arrival <= now:
                queue.append(pending.pop(0))
            # admission: FIFO, by footprint
            while queue and len(active) < self.max_active:
                j = queue[0]
                fp = self.ex.footprint(j.n)
                if fp > self.budget:
                    queue.pop(0)
                    j.error = "larger than the HBM budget"
                    j.finished_at = self.clock() - t0
                    rejected += 1
                    done.append(j)
                    continue
                if used + fp > self.budget or (active and inflight + j.n > self.max_particles):
                    break
                queue.pop(0)
                try:
                    self.ex.admit(j)
                except Exception as e:
                    j.error = f"admission failed: {e}"
                    j.finished_at = self.clock() - t0
                    done.append(j)
                    continue
                j.admitted_at = self.clock() - t0
                j.state["_fp"] = fp
                used += fp
                inflight += j.n
                active.append(j)
            if not active:
                if pending and realtime:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - (self.clock() - t0))))
                continue
            max_act = max(max_act, len(active))
            ts = self.clock()
            self.ex.step(active)
            tick_s.append(self.clock() - ts)
            ticks += 1
            solves += len(active)
            psolves += sum(j.n for j in active)
            still = []
            for j in active:
                if j.error is not None or j.done:
                    j.finished_at = self.clock() - t0
                    used -= j.state.get("_fp", 0)
                    inflight -= j.n
                    self.ex.release(j)
                    done.append(j)
                else:
                    still.append(j)
            active = still
        makespan = self.clock() - t0
        ok = [j for j in done if j.error is None]
        lat = [j.finished_at - j.arrival for j in ok]
        return Report(completed=len(ok), failed=len(done) - len(ok) - rejected, rejected=rejected,
                      makespan_s=makespan, latencies_s=lat, solves=solves,
                      particle_solves=psolves, max_active=max_act, ticks=ticks, tick_s=tick_s)


def jobs_from_stream(requests, steps: int = 4) -> List[Job]:
    """Jobs from requests carrying x, m, h, arrival and rid:
    dt = 1e-3 sqrt(R^3 / (G M)) with G = 1, R the 90%-mass radius and M the
    total mass of the system."""
    out = []
    for q in requests:
        r = np.linalg.norm(q.x - q.x.mean(0), axis=1)
        R = float(np.percentile(r, 90))
        M = float(q.m.sum())
        out.append(Job(rid=q.rid, arrival=q.arrival, n=len(q.m), steps=steps,
                       dt=1e-3 * math.sqrt(R ** 3 / M), payload=(q.x, q.m, q.h)))
    return out
