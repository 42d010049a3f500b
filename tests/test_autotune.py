"""Autotuner search and cache on the CPU, with a stand-in for the timing."""
import json

import pytest

from paper_2602_05804_amd import autotune


class _T:
    """Tensor stand-in: shape and device only."""

    def __init__(self, n):
        self.shape = (n,)
        self.device = "cpu"


def _cost(cfg):
    # separable bowl: best at leaf 12, near kernel 7, top depth 12
    c = abs(cfg["leaf_size"] - 12) + abs(cfg["near_kernel"] - 7) * 0.5
    c += abs(cfg.get("fp64_top_depth", 12) - 12) * 0.1
    return 1.0 + c


def test_search_finds_separable_minimum(monkeypatch):
    calls = []
    monkeypatch.setattr(autotune, "time_config",
                        lambda x, m, h, cfg, *a, **k: calls.append(dict(cfg)) or _cost(cfg))
    res = autotune.search(None, _T(1000), None, precision="fp32c")
    assert res["config"] == {"leaf_size": 12, "near_kernel": 7, "fp64_top_depth": 12}
    assert res["seconds"] == 1.0
    # a coordinate search: one run per value per axis, not the full product
    assert len(calls) == (1 + (len([k for k in autotune.LEAF_SIZES if k <= 16]) - 1)
                          + (len(autotune.NEAR_KERNELS["fp32c"]) - 1)
                          + (len(autotune.TOP_DEPTHS) - 1))
    # every shape tried is one the library accepts, and FP32C leaves stay <= 16
    assert all(c["near_kernel"] in (0, 1, 6, 7, 13) for c in calls)
    assert all(c["leaf_size"] <= 16 for c in calls)


def test_cache_roundtrip(monkeypatch, tmp_path):
    import torch

    monkeypatch.setattr(torch.cuda, "get_device_name", lambda d=None: "TestGPU")
    n_search = []

    def fake_search(x, m, h, theta, order, precision, log=None):
        n_search.append(1)
        return {"config": {"leaf_size": 8, "near_kernel": 6}, "seconds": 0.1}

    monkeypatch.setattr(autotune, "search", fake_search)
    path = str(tmp_path / "cache.json")
    c1 = autotune.tuned_config(_T(1000), _T(1000), _T(1000), label="plummer", cache_path=path)
    c2 = autotune.tuned_config(_T(1100), _T(1100), _T(1100), label="plummer", cache_path=path)
    assert c1 == c2 == {"leaf_size": 8, "near_kernel": 6}
    assert len(n_search) == 1  # same power-of-two bucket: cached
    autotune.tuned_config(_T(5000), _T(5000), _T(5000), label="plummer", cache_path=path)
    assert len(n_search) == 2  # another bucket
    keys = sorted(json.load(open(path)))
    assert len(keys) == 2 and all(k.startswith("TestGPU|N~") for k in keys)


@pytest.mark.gpu
def test_autotuned_solver_parity(orc):
    import numpy as np
    import torch

    import paper_2602_05804_amd as P
    import workloads

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    print("case: autotuned config parity", flush=True)
    x, m, h = workloads.plummer(20000, seed=3)
    xd, md, hd = (torch.from_numpy(a).cuda() for a in (x, m, h))
    res = autotune.search(xd, md, hd, reps=2)
    cfg = res["config"]
    assert cfg["leaf_size"] in autotune.LEAF_SIZES
    acc, pot = P.Solver(**cfg).solve(xd, md, hd)
    torch.cuda.synchronize()
    oa, op = orc.sfmm_solve(x, m, h, theta=0.5, leaf_size=cfg["leaf_size"])
    acc = acc.cpu().numpy()
    nb = np.linalg.norm(oa, axis=1)
    assert (np.linalg.norm(acc - oa, axis=1) / np.maximum(nb, 1e-6 * np.sqrt((nb ** 2).mean()))).max() < 1e-12


def test_bucket_lookup():
    tuned = {1024: {"leaf_size": 8}, 65536: {"leaf_size": 16, "near_kernel": 13}}
    assert autotune.bucket(1000) == 1024 and autotune.bucket(3000) == 4096
    assert autotune.config_for({}, 5000) == {}
    assert autotune.config_for(tuned, 700) == {"leaf_size": 8}
    assert autotune.config_for(tuned, 7000) == {"leaf_size": 8}  # log-nearer to 2^10 than 2^16
    assert autotune.config_for(tuned, 10 ** 6) == {"leaf_size": 16, "near_kernel": 13}
    # a copy: the caller may change it
    c = autotune.config_for(tuned, 10 ** 6)
    c["leaf_size"] = 4
    assert tuned[65536]["leaf_size"] == 16


def test_tune_buckets_one_search_per_bucket(monkeypatch):
    seen = []

    def fake_search(x, m, h, theta, order, precision, reps=3, log=None, base=None):
        seen.append(x)
        return {"config": {**(base or {}), "leaf_size": 8 if x < 5000 else 12, "near_kernel": 0},
                "seconds": 0.01}

    monkeypatch.setattr(autotune, "search", fake_search)
    out = autotune.tune_buckets([1000, 1100, 3000, 70000], lambda n: (n, None, None),
                                base={"walk": "level"})
    assert seen == [1024, 4096, 65536]
    assert out == {1024: {"leaf_size": 8, "near_kernel": 0},
                   4096: {"leaf_size": 8, "near_kernel": 0},
                   65536: {"leaf_size": 12, "near_kernel": 0}}
