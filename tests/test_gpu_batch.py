"""GPU: packed (forest) solves of several systems, the leapfrog update and
the serving loop.

A system solved inside a batch must get exactly what a solve of it alone
returns in FP64 (the same tree below its root, the same lists in the same
order, the same arithmetic), and agree to the FP32-compensated bound in
that form.  Systems overlap in space, so any interaction across systems
would show.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


@pytest.fixture(scope="module")
def P(torch):
    import paper_2602_05804_amd as P

    return P


def dev(torch, *arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def _systems():
    e = (np.zeros((0, 3)), np.zeros(0), np.zeros(0))
    one = (np.array([[0.3, -0.2, 0.1]]), np.array([1.5]), np.array([0.2]))
    dup = (np.zeros((30, 3)), np.full(30, 0.1), np.full(30, 0.05))
    x, m, h = workloads.plummer(2000, seed=15)
    far = (x + 1.0e3, m, h)
    return [e,
            workloads.plummer(3000, seed=11),
            workloads.plummer(12345, seed=12),
            e,
            workloads.polytrope(5000, seed=13),
            workloads.plummer(7, seed=14),
            one,
            dup,
            far]


@pytest.mark.parametrize("order,far", [(3, "leaf"), (1, "leaf"), (3, "shared")])
def test_batch_equals_alone_fp64(torch, P, order, far):
    print(f"case: batch vs alone fp64 order {order} far {far}", flush=True)
    systems = _systems()
    dsys = [tuple(dev(torch, *s)) for s in systems]
    s = P.Solver(far=far)
    res = s.solve_batch(dsys, theta=0.5, order=order)
    alone = P.Solver(far=far)
    for i, (xd, md, hd) in enumerate(dsys):
        a, p = alone.solve(xd, md, hd, theta=0.5, order=order)
        assert torch.equal(res[i][0], a), f"system {i}: acc differs from the solo solve"
        assert torch.equal(res[i][1], p), f"system {i}: pot differs from the solo solve"
    # the same context again with fewer, smaller systems
    sub = [dsys[5], dsys[1], dsys[0]]
    res2 = s.solve_batch(sub, theta=0.5, order=order)
    for (xd, md, hd), (a2, p2) in zip(sub, res2):
        a, p = alone.solve(xd, md, hd, theta=0.5, order=order)
        assert torch.equal(a2, a) and torch.equal(p2, p)


def test_batch_against_oracle(torch, P, orc):
    print("case: batch vs oracle", flush=True)
    systems = _systems()
    res = P.Solver().solve_batch([tuple(dev(torch, *s)) for s in systems], theta=0.5)
    for i in (1, 4, 5, 8):
        x, m, h = systems[i]
        oa, op = orc.sfmm_solve(x, m, h, theta=0.5)
        a = res[i][0].cpu().numpy(); p = res[i][1].cpu().numpy()
        nb = np.linalg.norm(oa, axis=1)
        assert (np.linalg.norm(a - oa, axis=1) / nb).max() < 1e-12
        assert (np.abs(p - op) / np.abs(op)).max() < 1e-12


def test_batch_fp32c(torch, P, orc):
    print("case: batch fp32c", flush=True)
    systems = _systems()
    res = P.Solver().solve_batch([tuple(dev(torch, *s)) for s in systems], theta=0.5,
                                 precision="fp32c")
    for i, (x, m, h) in enumerate(systems):
        a = res[i][0].cpu().numpy(); p = res[i][1].cpu().numpy()
        if len(m) == 0:
            assert a.shape == (0, 3)
            continue
        oa, op = orc.sfmm_solve(x, m, h, theta=0.5)
        nb = np.linalg.norm(oa, axis=1)
        if nb.max() == 0:
            assert np.all(a == 0)
        else:
            rel = np.linalg.norm(a - oa, axis=1) / nb
            assert np.sqrt((rel ** 2).mean()) <= 1e-6, f"system {i}"
        assert np.sqrt((((p - op) / op) ** 2).mean()) <= 1e-6


def test_batch_rejects_bad_offsets(torch, P):
    print("case: batch bad input", flush=True)
    s = P.Solver()
    x, m, h = dev(torch, *workloads.plummer(100, seed=3))
    with pytest.raises(P.SfmmError):
        s.solve_batch([(x, m, h), (x, m[:50], h)])
    with pytest.raises(P.SfmmError):
        P.Solver(walk="leaf").solve_batch([(x, m, h), (x, m, h)])


def test_leapfrog(torch, P):
    print("case: leapfrog", flush=True)
    rng = np.random.default_rng(4)
    x, v, a = (rng.standard_normal((1001, 3)) for _ in range(3))
    xd, vd, ad = dev(torch, x, v, a)
    P.leapfrog(xd, vd, ad, 0.25, 0.125)
    torch.cuda.synchronize()
    v1 = v + 0.25 * a
    x1 = x + 0.125 * v1
    assert np.array_equal(vd.cpu().numpy(), v1)
    assert np.array_equal(xd.cpu().numpy(), x1)


def test_serving_loop(torch, P):
    """Continuous batching on the GPU: every request completes, and a request
    that went through packed solves ends in the state a solo KDK integration
    of it reaches (bit for bit in FP64)."""
    print("case: serving loop", flush=True)
    from paper_2602_05804_amd import serve

    reqs = workloads.serving_stream(count=24, seed=9, rate=400.0, nmin=50, nmax=30000)
    jobs = serve.jobs_from_stream(reqs, steps=3)
    ref = {j.rid: (j.payload, j.dt) for j in jobs}
    # several packs per tick; systems above the cap are packs of their own
    ex = serve.GpuExecutor(pack_particles=20000)
    finals = {}
    orig_release = ex.release

    def keep(job):
        finals[job.rid] = job.state["x"].cpu().numpy()
        orig_release(job)

    ex.release = keep
    rep = serve.Server(ex, hbm_budget=ex.footprint(60000)).run(jobs)
    assert rep.completed == len(jobs) and rep.failed == 0 and rep.rejected == 0
    summ = rep.summary()
    assert summ["p99_latency_ms"] >= summ["p50_latency_ms"] > 0
    # solo KDK for two requests: one small (packed), one large
    for pick in (min(jobs, key=lambda j: j.n), max(jobs, key=lambda j: j.n)):
        (x, m, h), dt = ref[pick.rid]
        s = P.Solver()
        xd, md, hd = dev(torch, x, m, h)
        vd = torch.zeros_like(xd)
        acc, _ = s.solve(xd, md, hd)
        for k in range(1, 4):
            P.leapfrog(xd, vd, acc, 0.5 * dt if k == 1 else dt, dt)
            acc, _ = s.solve(xd, md, hd)
        P.leapfrog(xd, vd, acc, 0.5 * dt, 0.0)
        assert np.array_equal(xd.cpu().numpy(), finals[pick.rid])


def test_serving_loop_tuned(torch, P):
    """Serving with per-bucket tuned settings: every request completes, the
    packs use the Solver of their bucket, and a request larger than the pack
    cap (a pack of its own, nearest the 2^15 bucket) ends in the state a solo KDK
    integration with that bucket's settings reaches (bit for bit, FP64)."""
    print("case: serving loop with tuned buckets", flush=True)
    from paper_2602_05804_amd import serve

    reqs = workloads.serving_stream(count=16, seed=10, rate=400.0, nmin=50, nmax=30000)
    jobs = serve.jobs_from_stream(reqs, steps=2)
    ref = {j.rid: (j.payload, j.dt) for j in jobs}
    tuned = {1024: {"leaf_size": 6}, 32768: {"leaf_size": 16, "near_kernel": 13}}
    ex = serve.GpuExecutor(pack_particles=15000, tuned=tuned)
    finals = {}
    orig_release = ex.release

    def keep(job):
        finals[job.rid] = job.state["x"].cpu().numpy()
        orig_release(job)

    ex.release = keep
    rep = serve.Server(ex, hbm_budget=ex.footprint(60000)).run(jobs)
    assert rep.completed == len(jobs) and rep.failed == 0 and rep.rejected == 0
    used = set(ex._solvers)
    assert (("leaf_size", 16), ("near_kernel", 13)) in used
    big = max(jobs, key=lambda j: j.n)
    assert big.n > 15000
    (x, m, h), dt = ref[big.rid]
    s = P.Solver(leaf_size=16, near_kernel=13)
    xd, md, hd = dev(torch, x, m, h)
    vd = torch.zeros_like(xd)
    acc, _ = s.solve(xd, md, hd)
    for k in range(1, 3):
        P.leapfrog(xd, vd, acc, 0.5 * dt if k == 1 else dt, dt)
        acc, _ = s.solve(xd, md, hd)
    P.leapfrog(xd, vd, acc, 0.5 * dt, 0.0)
    assert np.array_equal(xd.cpu().numpy(), finals[big.rid])


def test_context_reuse_small_then_large(torch, P):
    """A context that solved a small system first sizes its list pools for a
    much larger one (the walk retries with grown pools)."""
    print("case: context reuse small -> large", flush=True)
    s = P.Solver()
    small = dev(torch, *workloads.plummer(300, seed=21))
    s.solve(*small)
    big = dev(torch, *workloads.plummer(60000, seed=22))
    a, p = s.solve(*big)
    a2, p2 = P.Solver().solve(*big)
    assert torch.equal(a, a2) and torch.equal(p, p2)
    sysl = [dev(torch, *workloads.plummer(n, seed=30 + n)) for n in (200, 5000, 20000, 7000)]
    t = P.Solver()
    t.solve(*small)
    res = t.solve_batch(sysl)
    for (xd, md, hd), (ab, pb) in zip(sysl, res):
        aa, pa = P.Solver().solve(xd, md, hd)
        assert torch.equal(ab, aa) and torch.equal(pb, pa)


def test_serving_failure_isolated(torch, P):
    """A request with a non-finite position fails alone; the other systems of
    its pack complete."""
    print("case: serving failure isolation", flush=True)
    from paper_2602_05804_amd import serve

    reqs = workloads.serving_stream(count=6, seed=4, rate=1e6, nmin=200, nmax=3000)
    jobs = serve.jobs_from_stream(reqs, steps=2)
    x, m, h = jobs[2].payload
    x = x.copy()
    x[5, 0] = np.nan
    jobs[2].payload = (x, m, h)
    ex = serve.GpuExecutor(pack_particles=10**7)
    rep = serve.Server(ex, hbm_budget=ex.footprint(10**6)).run(jobs, realtime=False)
    assert rep.completed == 5 and rep.failed == 1
    assert jobs[2].error is not None and "non-finite" in jobs[2].error


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-13), ("fp32c", 1e-6)])
def test_binary_momentum_drift(torch, P, precision, bound):
    """Gravity-only leapfrog of the binary polytrope: the pairwise forces
    keep the total momentum to rounding over many steps (without pressure the
    cold stars collapse, so energy is not a useful check here)."""
    print(f"case: binary leapfrog drift {precision}", flush=True)
    from paper_2602_05804_amd import sweep

    recs = list(sweep.binary(3000, 20, precision, "shared", 0.05, every=5))
    assert len(recs) == 4
    assert max(r["dP_rel"] for r in recs) < bound


def test_binary_leapfrog_follows_oracle(torch, P, orc):
    """A few kick-drift-kick steps of the binary polytrope (reduced N) with the
    device leapfrog and the GPU solve, against the same steps driven by the CPU
    oracle's solve in plain FP64 numpy: positions and velocities agree to
    1e-12 of their scale (the solver's workspace is reused from step to step)."""
    print("case: binary leapfrog vs oracle-driven KDK, 2 x 2000", flush=True)
    import workloads

    x, m, h, v = workloads.binary_polytrope(2000)
    dt = 0.02
    steps = 3
    s = P.Solver(include_self_potential=False)
    xd, md, hd, vd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (x, m, h, v))
    acc, _ = s.solve(xd, md, hd)
    for _ in range(steps):
        P.leapfrog(xd, vd, acc, 0.5 * dt, dt)
        acc, _ = s.solve(xd, md, hd)
        P.leapfrog(xd, vd, acc, 0.5 * dt, 0.0)
    torch.cuda.synchronize()
    xo, vo = x.copy(), v.copy()
    ao, _ = orc.sfmm_solve(xo, m, h, theta=0.5, include_self=False)
    for _ in range(steps):
        vo = vo + (0.5 * dt) * ao
        xo = xo + dt * vo
        ao, _ = orc.sfmm_solve(xo, m, h, theta=0.5, include_self=False)
        vo = vo + (0.5 * dt) * ao
    xs, vs = xd.cpu().numpy(), vd.cpu().numpy()
    assert np.abs(xs - xo).max() <= 1e-12 * np.abs(xo).max()
    assert np.abs(vs - vo).max() <= 1e-12 * np.abs(vo).max()
    s.close()
