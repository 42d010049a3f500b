"""Autotuner for the solve's free parameters: leaf size, the P2P and
P2P kernel shape and, in the FP32-compensated form, the depth above which
M2L stays in FP64.

A coordinate search on the caller's (or a synthetic) input: each parameter in
turn is swept with the others fixed at their best so far, timing the median
of a few solves.  The leaf size changes the tree and hence the result (within
the method's truncation error; the oracle accepts any leaf size, so parity
holds for every choice); the kernel shapes change only the summation order.

Results are cached in a JSON file keyed by (device name, N rounded to a power
of two, a distribution label, precision, theta, order), so a serving process
tunes once per class of request:

    cfg = autotune.tuned_config(x, m, h, label="polytrope")   # device tensors
    solver = Solver(**cfg)
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Optional

LEAF_SIZES = (6, 8, 10, 12, 16, 24, 32)
# the P2P shapes of sfmm_config.near_kernel worth a try per precision (the
# far field has one shape per mode)
NEAR_KERNELS = {"fp64": (0, 13, 6), "fp32c": (0, 6, 7)}
TOP_DEPTHS = (4, 8, 12, 128)  # 128: every M2L in FP64


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "sfmm_autotune.json")


def _key(device_name: str, n: int, label: str, precision: str, theta: float, order: int) -> str:
    return f"{device_name}|N~{bucket(n)}|{label}|{precision}|theta={theta:g}|p={order}"


def time_config(x, m, h, cfg: Dict, theta=0.5, order=3, precision="fp64", reps=5) -> float:
    """Median seconds of one solve with Solver(**cfg) (after one warm-up)."""
    import torch

    import paper_2602_05804_amd as sfmm

    s = sfmm.Solver(**cfg)
    try:
        s.solve(x, m, h, theta=theta, order=order, precision=precision)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            s.solve(x, m, h, theta=theta, order=order, precision=precision)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ts.sort()
        return ts[len(ts) // 2]
    finally:
        s.close()


def search(x, m, h, theta=0.5, order=3, precision="fp64", reps=5, log=None,
           leaf_sizes=LEAF_SIZES, base: Optional[Dict] = None) -> Dict:
    """Coordinate search; returns the best Solver keyword arguments and the
    time of every configuration tried.  `base` holds fixed Solver arguments
    (walk, far mode, ...); `leaf_sizes` = (k,) keeps the leaf size at k."""
    base = dict(base or {})
    if precision == "fp32c":  # the FP32-compensated kernels take leaves of at most 16
        leaf_sizes = tuple(k for k in leaf_sizes if k <= 16) or (10,)
    best = {**base, "leaf_size": 10 if 10 in leaf_sizes else leaf_sizes[0], "near_kernel": 0}
    if precision == "fp32c":
        best["fp64_top_depth"] = 8
    tried = []

    def run(cfg):
        t = time_config(x, m, h, cfg, theta, order, precision, reps)
        tried.append({**cfg, "seconds": t})
        if log:
            log(f"autotune {cfg}: {t * 1e3:.3f} ms")
        return t

    axes = [("leaf_size", tuple(leaf_sizes)), ("near_kernel", NEAR_KERNELS[precision])]
    if precision == "fp32c":
        axes.append(("fp64_top_depth", TOP_DEPTHS))
    t_best = run(dict(best))
    for name, values in axes:
        for v in values:
            if v == best[name]:
                continue
            cfg = dict(best, **{name: v})
            t = run(cfg)
            if t < t_best:
                best, t_best = cfg, t
    return {"config": best, "seconds": t_best, "tried": tried}


def bucket(n: int) -> int:
    """The power of two nearest to n (on a log scale): the size class the
    cache and the serving loop tune for."""
    return 2 ** round(math.log2(max(n, 1)))


def config_for(tuned: Dict[int, Dict], n: int) -> Dict:
    """The tuned Solver arguments for a solve of n particles: those of the
    tuned bucket nearest to n on a log scale ({} when nothing is tuned)."""
    if not tuned:
        return {}
    b = min(tuned, key=lambda k: (abs(math.log2(k) - math.log2(max(n, 1))), k))
    return dict(tuned[b])


def tune_buckets(sizes, make_input, theta=0.5, order=3, precision="fp64", reps=3, log=None,
                 base: Optional[Dict] = None) -> Dict[int, Dict]:
    """Tuned Solver arguments per size bucket: one search per distinct
    bucket of `sizes`, on the input make_input(n) returns (device x, m, h)."""
    out = {}
    for b in sorted({bucket(n) for n in sizes}):
        x, m, h = make_input(b)
        res = search(x, m, h, theta, order, precision, reps=reps, log=log, base=base)
        cfg = {k: v for k, v in res["config"].items() if k not in (base or {})}
        out[b] = cfg
        if log:
            log(f"autotune bucket N~{b}: {cfg} ({res['seconds'] * 1e3:.3f} ms)")
    return out


def tuned_config(x, m, h, label: str = "default", theta=0.5, order=3, precision="fp64",
                 cache_path: Optional[str] = None, retune: bool = False, log=None) -> Dict:
    """Solver keyword arguments for this input class, from the cache or a new
    search (whose result is then stored)."""
    import torch

    path = cache_path or default_cache_path()
    key = _key(torch.cuda.get_device_name(x.device), int(m.shape[0]), label, precision, theta,
               order)
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    if not retune and key in cache:
        return dict(cache[key]["config"])
    res = search(x, m, h, theta, order, precision, log=log)
    cache[key] = {"config": res["config"], "seconds": res["seconds"]}
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return dict(res["config"])
