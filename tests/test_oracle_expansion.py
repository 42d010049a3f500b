"""Pins of the oracle's multipole machinery.

* D_alpha = d^alpha (1/|r|) against sympy's symbolic derivatives and
  Laplace's equation (Sect. 2.1 defines D_n as the n-th gradient of 1/|r|).
* M2L + L2P (Sect. 2.2, Eq. dmkdeffmm and the M_k definition) against the
  direct sum: exact for point masses at both centres, monopole limit at p=0,
  and Taylor-remainder convergence ~ (l/d)^(p+1) for p = 0..5.
* Newton's third law for one node pair (the reason SFMM conserves momentum,
  Sect. 2.2 end).
"""
import numpy as np
import pytest
import sympy as sp


def test_multi_index_order(orc):
    mi = orc.multi_indices(4)
    assert len(mi) == 35
    assert mi[0].tolist() == [0, 0, 0]
    deg = mi.sum(1)
    assert np.all(np.diff(deg) >= 0)
    assert len({tuple(a) for a in mi}) == 35


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_derivs_match_sympy(orc, seed):
    X, Y, Z = sp.symbols("x y z", real=True)
    f = 1 / sp.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    rng = np.random.default_rng(seed)
    r = rng.normal(size=3)
    order = 6
    D = orc.derivs(order, r)
    for k, (a, b, c) in enumerate(orc.multi_indices(order)):
        expr = f
        if a: expr = sp.diff(expr, X, a)
        if b: expr = sp.diff(expr, Y, b)
        if c: expr = sp.diff(expr, Z, c)
        val = float(expr.subs({X: r[0], Y: r[1], Z: r[2]}))
        assert D[k] == pytest.approx(val, rel=1e-12, abs=1e-12 * np.abs(D).max())


def test_derivs_laplace(orc):
    r = np.array([0.3, -1.1, 0.7])
    order = 7
    D = orc.derivs(order, r)
    mi = orc.multi_indices(order)
    idx = {tuple(a): k for k, a in enumerate(mi)}
    for a in mi:
        if a.sum() + 2 > order:
            continue
        s = 0.0
        for c in range(3):
            b = a.copy(); b[c] += 2
            s += D[idx[tuple(b)]]
        scale = max(abs(D[idx[tuple(a)]]), 1.0) * np.linalg.norm(r) ** -(a.sum() + 3)
        assert abs(s) < 1e-12 * max(scale, 1.0)


def _direct_unsoftened(xs, ms, xt):
    acc = np.zeros((len(xt), 3)); pot = np.zeros(len(xt))
    for i, xi in enumerate(xt):
        d = xs - xi
        r = np.linalg.norm(d, axis=1)
        acc[i] = (ms[:, None] * d / r[:, None] ** 3).sum(0)
        pot[i] = -(ms / r).sum()
    return acc, pot


@pytest.mark.parametrize("p", [0, 1, 3, 5])
def test_point_masses_at_centres_are_exact(orc, p):
    sS = np.array([2.0, -1.0, 0.5]); sT = np.array([-0.3, 0.4, 0.1])
    acc, pot = orc.m2l_pair(p, sS[None], np.array([0.8]), sS, sT[None], sT)
    a_ref, p_ref = _direct_unsoftened(sS[None], np.array([0.8]), sT[None])
    assert acc[0] == pytest.approx(a_ref[0], rel=1e-14)
    assert pot[0] == pytest.approx(p_ref[0], rel=1e-14)


def test_monopole_limit(orc):
    rng = np.random.default_rng(3)
    xs = rng.normal(scale=0.1, size=(20, 3)) + [3.0, 0.0, 0.0]
    ms = rng.uniform(0.5, 1.5, 20)
    sS = (ms[:, None] * xs).sum(0) / ms.sum()
    sT = np.zeros(3)
    xt = rng.normal(scale=0.1, size=(5, 3))
    acc, pot = orc.m2l_pair(0, xs, ms, sS, xt, sT)
    r = sS - sT
    mono = ms.sum() * r / np.linalg.norm(r) ** 3
    for a in acc:
        assert a == pytest.approx(mono, rel=1e-14)
    assert pot == pytest.approx(-ms.sum() / np.linalg.norm(r), rel=1e-14)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_taylor_remainder_convergence(orc, p):
    rng = np.random.default_rng(10 + p)
    us = rng.uniform(-1, 1, size=(40, 3)); ut = rng.uniform(-1, 1, size=(30, 3))
    ms = rng.uniform(0.5, 1.5, 40)
    d = np.array([1.0, 0.6, -0.4]) / np.linalg.norm([1.0, 0.6, -0.4])
    errs = []
    for l in (0.08, 0.04, 0.02):
        xs = 10.0 * d + l * us
        sS = (ms[:, None] * xs).sum(0) / ms.sum()
        xt = l * ut
        sT = xt.mean(0)
        acc, pot = orc.m2l_pair(p, xs, ms, sS, xt, sT)
        a_ref, p_ref = _direct_unsoftened(xs, ms, xt)
        errs.append(np.abs(acc - a_ref).max() / np.abs(a_ref).max())
    for e0, e1 in zip(errs[:-1], errs[1:]):
        ratio = e0 / e1
        # halving the node size divides the remainder by ~2^(p+1)
        assert 2 ** (p + 1) * 0.6 < ratio < 2 ** (p + 1) * 1.6, (errs, ratio)


def test_node_pair_third_law(orc):
    rng = np.random.default_rng(5)
    xa = rng.normal(scale=0.3, size=(30, 3)); ma = rng.uniform(0.5, 1.5, 30)
    xb = rng.normal(scale=0.3, size=(25, 3)) + [4.0, 1.0, -2.0]; mb = rng.uniform(0.5, 1.5, 25)
    sa = (ma[:, None] * xa).sum(0) / ma.sum()
    sb = (mb[:, None] * xb).sum(0) / mb.sum()
    for p in (1, 3, 5):
        acc_a, _ = orc.m2l_pair(p, xb, mb, sb, xa, sa)
        acc_b, _ = orc.m2l_pair(p, xa, ma, sa, xb, sb)
        Fa = (ma[:, None] * acc_a).sum(0); Fb = (mb[:, None] * acc_b).sum(0)
        assert np.abs(Fa + Fb).max() < 1e-14 * np.abs(Fa).max()
