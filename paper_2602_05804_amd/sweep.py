"""Accuracy and scaling sweeps of the GPU SFMM solve (the SFMM half of the
paper's Plummer / homogeneous-sphere tests, Sect. 4.1).

  python -m paper_2602_05804_amd.sweep accuracy  [--n 100000]
      for theta in 0.10, 0.15, ..., 0.60: per-particle relative acceleration
      error |a - a_direct| / |a_direct| (mean, max, 10th and 90th
      percentiles) against the softened direct sum on the GPU, for a Plummer
      sphere and a homogeneous sphere, and the time of one solve
  python -m paper_2602_05804_amd.sweep scaling   [--theta 0.5]
      time of one solve of a Plummer sphere for N = 1e4 ... 3e6
  python -m paper_2602_05804_amd.sweep binary    [--n-each 100000 --steps 200]
      gravity-only leapfrog evolution of the binary polytrope (Sect. 4.2's
      binary without the gas dynamics): drift of the linear momentum, angular
      momentum and energy

Prints one JSON object per line.  Inputs are the seeded generators of the
`workloads` module (Plummer a = 1, M = 1, seed 1; homogeneous sphere R = 1,
M = 1, seed 11; h = 1.2 (m / rho)^(1/3) from the analytic density).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def _timed_solve(solver, xd, md, hd, theta, precision, reps=5):
    import torch

    acc, pot = solver.solve(xd, md, hd, theta=theta, precision=precision)  # warm-up
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        acc, pot = solver.solve(xd, md, hd, theta=theta, precision=precision)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return acc, pot, float(np.median(ts))


def accuracy(n: int, precision: str, far: str):
    import torch

    import paper_2602_05804_amd as sfmm
    import workloads

    thetas = [round(0.10 + 0.05 * k, 2) for k in range(11)]
    for name, gen in (("plummer", lambda: workloads.plummer(n, seed=1)),
                      ("homogeneous", lambda: workloads.homogeneous_sphere(n, seed=11))):
        x, m, h = gen()
        xd, md, hd = (torch.from_numpy(a).cuda() for a in (x, m, h))
        s = sfmm.Solver(far=far)
        da, dp = s.direct(xd, md, hd)
        torch.cuda.synchronize()
        da = da.cpu().numpy()
        dn = np.linalg.norm(da, axis=1)
        for th in thetas:
            acc, pot, t = _timed_solve(s, xd, md, hd, th, precision)
            e = np.linalg.norm(acc.cpu().numpy() - da, axis=1) / dn
            st = s.stats()
            print(json.dumps({
                "sweep": "accuracy", "workload": name, "N": n, "theta": th,
                "precision": precision, "far": far,
                "err_mean": float(e.mean()), "err_max": float(e.max()),
                "err_p10": float(np.percentile(e, 10)), "err_p90": float(np.percentile(e, 90)),
                "pot_err_mean": float(np.mean(np.abs(pot.cpu().numpy() - dp.cpu().numpy())
                                              / np.abs(dp.cpu().numpy()))),
                "solve_ms": t * 1e3, "n_m2l_unique": st["n_m2l_unique"],
                "n_p2p_pairs": st["n_p2p_pairs"]}), flush=True)
        s.close()


def scaling(theta: float, precision: str, far: str, sizes):
    import torch

    import paper_2602_05804_amd as sfmm
    import workloads

    s = sfmm.Solver(far=far)
    for n in sizes:
        x, m, h = workloads.plummer(n, seed=1)
        xd, md, hd = (torch.from_numpy(a).cuda() for a in (x, m, h))
        _, _, t = _timed_solve(s, xd, md, hd, theta, precision)
        st = s.stats()
        print(json.dumps({
            "sweep": "scaling", "workload": "plummer", "N": n, "theta": theta,
            "precision": precision, "far": far, "solve_ms": t * 1e3,
            "particles_per_s": n / t, "max_depth": st["max_depth"],
            "n_m2l_unique": st["n_m2l_unique"], "n_p2p_pairs": st["n_p2p_pairs"]}), flush=True)
    s.close()


def binary(n_each: int, steps: int, precision: str, far: str, orbit_fraction: float,
           every: int = 0):
    """Gravity-only kick-drift-kick evolution of the binary polytrope (two
    n = 1.5 stars of M = 1 at separation 3R on a circular orbit): linear
    momentum P = sum m v, angular momentum L = sum m x cross v and energy
    E = sum m v^2 / 2 + sum m phi / 2 (no self term), relative to their
    initial values, every `every` steps (default: ten records); yields dicts."""
    import torch

    import paper_2602_05804_amd as sfmm
    import workloads

    x, m, h, v = workloads.binary_polytrope(n_each)
    xd, md, hd, vd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (x, m, h, v))
    s = sfmm.Solver(far=far, include_self_potential=False)
    period = 2.0 * np.pi * np.sqrt(27.0 / 2.0)
    dt = orbit_fraction * period / steps
    mcol = md[:, None]

    def invariants(acc, pot):
        p = (mcol * vd).sum(0)
        lv = (mcol * torch.cross(xd, vd, dim=1)).sum(0)
        e = 0.5 * (md * (vd * vd).sum(1)).sum() + 0.5 * (md * pot).sum()
        pabs = (md * vd.norm(dim=1)).sum()
        return p.cpu().numpy(), lv.cpu().numpy(), float(e), float(pabs)

    acc, pot = s.solve(xd, md, hd, precision=precision)
    p0, l0, e0, pabs = invariants(acc, pot)
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        sfmm.leapfrog(xd, vd, acc, 0.5 * dt, dt)
        acc, pot = s.solve(xd, md, hd, precision=precision)
        sfmm.leapfrog(xd, vd, acc, 0.5 * dt, 0.0)
        if k % (every or max(1, steps // 10)) == 0 or k == steps:
            p, lv, e, _ = invariants(acc, pot)
            yield {"sweep": "binary", "N": 2 * n_each, "step": k, "dt": dt,
                   "precision": precision, "far": far,
                   "dP_rel": float(np.linalg.norm(p - p0) / pabs),
                   "dL_rel": float(np.linalg.norm(lv - l0) / np.linalg.norm(l0)),
                   "dE_rel": abs(e - e0) / abs(e0), "seconds": time.perf_counter() - t0}
    s.close()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["accuracy", "scaling", "binary"])
    ap.add_argument("--n-each", type=int, default=100_000)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--orbit-fraction", type=float, default=0.25)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--precision", choices=["fp64", "fp32c"], default="fp64")
    ap.add_argument("--far", choices=["shared", "leaf"], default="shared")
    ap.add_argument("--sizes", type=str, default="10000,30000,100000,300000,1000000,3000000")
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    if args.what == "accuracy":
        accuracy(args.n, args.precision, args.far)
    elif args.what == "binary":
        for rec in binary(args.n_each, args.steps, args.precision, args.far, args.orbit_fraction):
            print(json.dumps(rec), flush=True)
    else:
        scaling(args.theta, args.precision, args.far, [int(v) for v in args.sizes.split(",")])


if __name__ == "__main__":
    main()
