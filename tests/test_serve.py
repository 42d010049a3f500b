"""Serving loop on the CPU with a stand-in executor: admission by footprint
in FIFO order, slot release, rejection of oversized requests and failure
isolation."""
import math

import numpy as np

from paper_2602_05804_amd import serve


def _jobs(ns, steps=3, gap=0.0):
    st = steps if callable(steps) else (lambda i: steps)
    return [serve.Job(rid=i, arrival=i * gap, n=n, steps=st(i), dt=1e-3)
            for i, n in enumerate(ns)]


def test_all_complete_within_budget():
    rng = np.random.default_rng(0)
    ns = [int(x) for x in 10 ** rng.uniform(2, 4, 40)]
    ex = serve.FakeExecutor(sec_per_particle=0.0, bytes_per_particle=10)
    budget = 10 * 30000
    rep = serve.Server(ex, hbm_budget=budget).run(_jobs(ns, steps=lambda i: 1 + i % 4),
                                                  realtime=False)
    assert rep.completed == 40 and rep.failed == 0 and rep.rejected == 0
    sizes = dict(enumerate(ns))
    for tick in ex.ticks:
        assert sum(sizes[r] for r in tick) * 10 <= budget
    # every job takes steps + 1 solves
    assert rep.solves == sum(2 + i % 4 for i in range(40))
    # FIFO: admission order follows arrival order
    first = {}
    for t, tick in enumerate(ex.ticks):
        for r in tick:
            first.setdefault(r, t)
    order = sorted(first, key=lambda r: (first[r], r))
    assert order == sorted(order)
    # continuous batching: some tick runs a request admitted earlier beside
    # one that joined when another request finished
    assert any(first[a] < t == first[b] > 0 for t, tick in enumerate(ex.ticks)
               for a in tick for b in tick)


def test_slots_and_max_active():
    ex = serve.FakeExecutor(sec_per_particle=0.0, bytes_per_particle=1)
    rep = serve.Server(ex, hbm_budget=1e12, max_active=3).run(_jobs([100] * 10, steps=2),
                                                              realtime=False)
    assert rep.completed == 10 and rep.max_active == 3
    assert max(len(t) for t in ex.ticks) == 3


def test_oversized_rejected_without_blocking():
    ex = serve.FakeExecutor(sec_per_particle=0.0, bytes_per_particle=1)
    rep = serve.Server(ex, hbm_budget=1000).run(_jobs([10, 5000, 20, 30]), realtime=False)
    assert rep.rejected == 1 and rep.completed == 3
    assert all(1 not in t for t in ex.ticks)


def test_failure_isolated():
    ex = serve.FakeExecutor(sec_per_particle=0.0, bytes_per_particle=1, fail_rid=2)
    rep = serve.Server(ex, hbm_budget=1e9).run(_jobs([50] * 6), realtime=False)
    assert rep.completed == 5 and rep.failed == 1
    # the failed request leaves after its first tick, the others keep going
    assert 2 in ex.ticks[0] and all(2 not in t for t in ex.ticks[1:])


def test_realtime_latency():
    ex = serve.FakeExecutor(sec_per_particle=1e-7, bytes_per_particle=1)
    rep = serve.Server(ex, hbm_budget=1e9).run(_jobs([1000] * 8, steps=2, gap=0.002))
    s = rep.summary()
    assert s["completed"] == 8
    assert 0 < s["p50_latency_ms"] <= s["p99_latency_ms"]
    assert math.isfinite(s["particles_per_s"]) and s["particles_per_s"] > 0


def test_jobs_from_stream():
    import workloads

    reqs = workloads.serving_stream(count=6, seed=3, nmin=100, nmax=2000)
    jobs = serve.jobs_from_stream(reqs, steps=2)
    assert [j.rid for j in jobs] == [q.rid for q in reqs]
    assert all(j.dt > 0 and j.n == len(q.m) for j, q in zip(jobs, reqs))
    assert all(a.arrival <= b.arrival for a, b in zip(jobs, jobs[1:]))


def test_max_particles_in_flight():
    ex = serve.FakeExecutor(sec_per_particle=0.0, bytes_per_particle=1)
    ns = [400, 300, 500, 200, 600, 100]
    rep = serve.Server(ex, hbm_budget=1e12, max_particles=1000).run(_jobs(ns, steps=1),
                                                                    realtime=False)
    assert rep.completed == len(ns)
    sizes = dict(enumerate(ns))
    assert all(sum(sizes[r] for r in t) <= 1000 for t in ex.ticks)
    # a request larger than the cap still runs (alone)
    ex = serve.FakeExecutor(sec_per_particle=0.0, bytes_per_particle=1)
    rep = serve.Server(ex, hbm_budget=1e12, max_particles=1000).run(_jobs([5000, 10]),
                                                                    realtime=False)
    assert rep.completed == 2 and ex.ticks[0] == [0]


class _Err(RuntimeError):
    def __init__(self, msg, code):
        super().__init__(msg)
        self.code = code


def _packs_run(fail):
    """solve_packs over two packs; `fail(kind, rid)` returns a status code to
    raise with, or None."""
    jobs = _jobs([10, 20, 30, 40])
    packs = [jobs[:2], jobs[2:]]
    results, errors = {}, {}

    def solve_pack(pack):
        for j in pack:
            c = fail("pack", j.rid)
            if c is not None:
                raise _Err(f"pack with {j.rid}", c)
        return [f"packed {j.rid}" for j in pack]

    def solve_one(j):
        c = fail("one", j.rid)
        if c is not None:
            raise _Err(f"alone {j.rid}", c)
        return f"alone {j.rid}"

    serve.solve_packs(packs, solve_pack, solve_one, lambda j, r: results.__setitem__(j.rid, r),
                      lambda j, m: errors.__setitem__(j.rid, m))
    return results, errors


def test_pack_failure_isolated_for_recoverable_codes():
    # EINVAL / ENONFINITE / ENOMEM / EUNSUPPORTED: the pack is re-solved system
    # by system and only the failing system fails
    for code in (-1, -2, -4, -5):
        res, err = _packs_run(lambda kind, rid: code if rid == 3 else None)
        assert res == {0: "packed 0", 1: "packed 1", 2: "alone 2"} and list(err) == [3]


def test_pack_device_error_ends_the_run():
    # a HIP error (EDEVICE) is not retried on the device: DeviceFault at once,
    # from the packed solve or from a retry
    import pytest

    with pytest.raises(serve.DeviceFault):
        _packs_run(lambda kind, rid: -3 if rid == 2 else None)
    with pytest.raises(serve.DeviceFault):
        _packs_run(lambda kind, rid: (-1 if kind == "pack" else -3) if rid == 1 else None)
    # an error without a status code is treated the same way
    with pytest.raises(serve.DeviceFault):
        _packs_run(lambda kind, rid: 0 if rid == 0 else None)
