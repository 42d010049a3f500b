"""Pins of the whole oracle solve.

* theta -> 0, or softening kernels larger than the system: every pair is
  summed directly, so SFMM must equal the softened direct sum of
  Eq. (softdirectsum) up to summation order;
* Newton's third law: |sum m a| / sum |m a| at rounding level (the paper's
  SFMM keeps linear momentum below 1e-13, Results);
* the per-leaf walk with the L2L chain (Algorithm 1), the recursive mutual
  traversal and direct evaluation of every ancestor's expansion agree (L2L of
  Eq. gravmtranslat re-centres a polynomial exactly);
* truncation error falls with theta and with p;
* Plummer closed forms: potential energy -3 pi G M^2 / (32 a) and the radial
  field -G M r / (r^2 + a^2)^(3/2), within the sampling noise.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_claims.json")))


def rel_err(a, b):
    nb = np.linalg.norm(b, axis=1)
    floor = 1e-6 * np.sqrt((nb ** 2).mean())
    return np.linalg.norm(a - b, axis=1) / np.maximum(nb, floor)


@pytest.fixture(scope="module")
def c1():
    return workloads.plummer(4096, seed=1)


@pytest.fixture(scope="module")
def c1_direct(orc, c1):
    x, m, h = c1
    return orc.direct(x, m, h)


def test_theta_to_zero_is_direct(orc, c1, c1_direct):
    x, m, h = c1
    acc, pot = orc.sfmm_solve(x, m, h, theta=1e-9)
    ad, pd = c1_direct
    assert rel_err(acc, ad).max() < 1e-13
    assert np.abs(pot - pd).max() < 1e-13 * np.abs(pd).max()


def test_large_softening_is_direct(orc):
    x, m, h = workloads.plummer(1000, seed=9)
    h = np.full(1000, 1e3)
    acc, pot = orc.sfmm_solve(x, m, h, theta=0.9)
    ad, pd = orc.direct(x, m, h)
    assert rel_err(acc, ad).max() < 1e-12
    assert np.abs(pot - pd).max() < 1e-13 * np.abs(pd).max()


def test_momentum(orc, c1):
    x, m, h = c1
    for theta in (0.3, 0.5, 0.7):
        acc, _ = orc.sfmm_solve(x, m, h, theta=theta)
        F = m[:, None] * acc
        res = np.linalg.norm(F.sum(0)) / np.abs(F).sum()
        assert res <= 1e-14
        assert res <= GOLD["momentum_conservation_bound"]["value"]


def test_modes_agree(orc, c1):
    x, m, h = c1
    t = orc.Tree(x, m, h, leaf_size=10, order=3)
    a0, p0, s0 = t.solve(0.5, mode=orc.MODE_PER_LEAF)
    a1, p1, _ = t.solve(0.5, mode=orc.MODE_MUTUAL)
    a2, p2, _ = t.solve(0.5, mode=orc.MODE_DIRECT_ANC)
    assert rel_err(a1, a0).max() < 1e-12
    assert rel_err(a2, a0).max() < 1e-12
    assert np.abs(p1 - p0).max() < 1e-13 * np.abs(p0).max()
    assert np.abs(p2 - p0).max() < 1e-13 * np.abs(p0).max()
    assert s0["n_m2l"] > 0 and s0["n_leaves_done"] == t.num_leaves


def test_targets_subset_is_bitwise(orc, c1):
    x, m, h = c1
    t = orc.Tree(x, m, h, leaf_size=10, order=3)
    a, p, _ = t.solve(0.5)
    tg = np.array([5, 4095, 17, 17, 2000])
    at, pt, st = t.solve(0.5, targets=tg)
    assert np.array_equal(at, a[tg]) and np.array_equal(pt, p[tg])
    assert st["n_leaves_done"] <= 4


def test_error_falls_with_theta_and_order(orc, c1, c1_direct):
    x, m, h = c1
    ad, _ = c1_direct
    t3 = orc.Tree(x, m, h, leaf_size=10, order=3)
    errs_theta = [rel_err(t3.solve(th)[0], ad).mean() for th in (0.3, 0.5, 0.7)]
    assert errs_theta[0] < errs_theta[1] < errs_theta[2]
    assert errs_theta[1] < 1e-3  # mean relative error at theta = 0.5, p = 3
    errs_p = []
    for p in (1, 2, 3, 4, 5):
        tp = orc.Tree(x, m, h, leaf_size=10, order=p)
        errs_p.append(rel_err(tp.solve(0.5)[0], ad).mean())
    assert all(e1 < e0 for e0, e1 in zip(errs_p[:-1], errs_p[1:])), errs_p


def test_plummer_closed_forms(orc):
    n = 20000
    x, m, h = workloads.plummer(n, seed=12)
    acc, pot = orc.sfmm_solve(x, m, h, theta=0.5, include_self=False)
    W = 0.5 * (m * pot).sum()
    assert W == pytest.approx(-3.0 * math.pi / 32.0, rel=0.03)
    r = np.linalg.norm(x, axis=1)
    ar = (acc * x).sum(1) / r
    for lo, hi in ((0.5, 0.8), (0.8, 1.2), (1.2, 2.0), (2.0, 4.0)):
        sel = (r > lo) & (r < hi)
        model = -r[sel] / (r[sel] ** 2 + 1.0) ** 1.5
        assert ar[sel].mean() == pytest.approx(model.mean(), rel=0.03)


def test_edge_cases(orc):
    # one particle: no force, potential is the self term only
    acc, pot = orc.sfmm_solve(np.array([[0.1, 0.2, 0.3]]), [2.0], [0.5], theta=0.5)
    assert np.all(acc == 0.0) and pot[0] == pytest.approx(-2.0 * 1.4 / 0.5)
    # coincident particles: zero pair force, pot = each other's psi(0, h) plus self
    x = np.zeros((12, 3)); m = np.full(12, 0.5); h = np.full(12, 0.1)
    acc, pot = orc.sfmm_solve(x, m, h, theta=0.5, leaf_size=4)
    assert np.all(acc == 0.0)
    assert pot == pytest.approx(np.full(12, -12 * 0.5 * 1.4 / 0.1))
    # two particles far apart: plain Newton
    x = np.array([[0.0, 0, 0], [3.0, 0, 0]])
    acc, pot = orc.sfmm_solve(x, [1.0, 2.0], [0.1, 0.1], theta=0.5, leaf_size=1,
                              include_self=False)
    assert acc[0] == pytest.approx([2.0 / 9.0, 0, 0], rel=1e-14)
    assert acc[1] == pytest.approx([-1.0 / 9.0, 0, 0], rel=1e-14)


def test_direct_targets_rows_equal_full_direct(orc):
    """The subset path of the direct sum (Eq. softdirectsum for listed targets)
    gives, row for row and bit for bit, the full direct sum's rows of those
    particles: any index, repeated indices, first and last particle, in the
    order given; an index outside [0, n) is an error."""
    import pytest

    x, m, h = workloads.plummer(700, seed=21)
    h[5] = 50.0  # one particle whose kernel covers every other
    acc, pot = orc.direct(x, m, h)
    rng = np.random.default_rng(5)
    tg = np.concatenate([[699, 0, 5], rng.integers(0, 700, 40), [5, 699]]).astype(np.int64)
    for include_self in (True, False):
        fa, fp = orc.direct(x, m, h, include_self=include_self)
        ta, tp = orc.direct(x, m, h, include_self=include_self, targets=tg)
        assert ta.shape == (len(tg), 3) and tp.shape == (len(tg),)
        assert np.array_equal(ta, fa[tg]) and np.array_equal(tp, fp[tg])
    assert np.array_equal(orc.direct(x, m, h, targets=tg)[0], acc[tg])
    for bad in ([700], [-1], [3, 700]):
        with pytest.raises(Exception):
            orc.direct(x, m, h, targets=np.array(bad, dtype=np.int64))


def test_parallel_per_leaf_equals_serial(orc):
    """Algorithm 1's loop over leaves on several threads (each leaf writes only
    its own particles, in the serial order) gives the serial result bit for
    bit, with the same interaction counts."""
    x, m, h = workloads.polytrope(6000, seed=8)
    t = orc.Tree(x, m, h, leaf_size=10, order=3)
    a1, p1, s1 = t.solve(0.5)
    a2, p2, s2 = t.solve_parallel(0.5, nthreads=4)
    assert s2["threads"] >= 1
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)
    assert (s1["n_m2l"], s1["n_p2p_pairs"], s1["n_leaves_done"]) == \
        (s2["n_m2l"], s2["n_p2p_pairs"], s2["n_leaves_done"])
