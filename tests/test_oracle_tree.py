"""Pins of the oracle's tree: keys, split rule, geometry and mass moments.

The tree type is free (the paper's kd-tree is replaced by a Morton binary
radix tree); these tests fix the properties every part of it must have,
checked by brute force on small inputs, and the mass moments of Eq. (massmom)
against closed forms and the translation identity of Eq. (massmomtrans).
"""
import math

import numpy as np
import pytest

import workloads


def test_keys_hand_values(orc):
    # bounding box [0,1]^3 (the corner points fix it)
    x = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.5, 0.0, 0.0], [0.0, 0.5, 0.0],
                  [0.0, 0.0, 0.5], [0.25, 0.0, 0.0]])
    n = len(x)
    t = orc.Tree(x, np.ones(n), np.ones(n), leaf_size=1, order=1)
    keys = t.keys(); perm = t.perm()
    k = dict(zip(perm.tolist(), keys.tolist()))
    assert k[0] == 0
    assert k[1] == 2 ** 63 - 1          # every cell clamped to 2^21 - 1
    assert k[2] == 1 << 62              # x's top bit is bit 62
    assert k[3] == 1 << 61              # then y
    assert k[4] == 1 << 60              # then z
    assert k[5] == 1 << 59              # x's second bit


def test_sort_is_stable_on_equal_keys(orc):
    x = np.zeros((7, 3))
    t = orc.Tree(x, np.ones(7), np.ones(7), leaf_size=2, order=1)
    assert t.perm().tolist() == list(range(7))
    assert np.all(t.keys() == 0)


def _check_tree(orc, x, m, h, leaf_size):
    t = orc.Tree(x, m, h, leaf_size=leaf_size, order=3)
    n = len(m)
    keys = t.keys(); perm = t.perm()
    assert sorted(perm.tolist()) == list(range(n))
    assert np.all(keys[:-1] <= keys[1:])
    eq = keys[:-1] == keys[1:]
    assert np.all(perm[:-1][eq] < perm[1:][eq])
    nd = t.nodes()
    lo, hi, L, R = nd["lo"], nd["hi"], nd["left"], nd["right"]
    assert lo[0] == 0 and hi[0] == n
    xs = x[perm]; ms = m[perm]; hs = h[perm]
    for i in range(t.num_nodes):
        cnt = hi[i] - lo[i]
        assert cnt >= 1
        if L[i] < 0:
            assert R[i] < 0 and cnt <= leaf_size
        else:
            assert cnt > leaf_size
            assert lo[L[i]] == lo[i] and hi[L[i]] == lo[R[i]] and hi[R[i]] == hi[i]
            assert nd["depth"][L[i]] == nd["depth"][i] + 1
            a, b = int(keys[lo[i]]), int(keys[hi[i] - 1])
            if a != b:
                bit = (a ^ b).bit_length() - 1
                left_bits = [(int(k) >> bit) & 1 for k in keys[lo[i]:hi[L[i]]]]
                right_bits = [(int(k) >> bit) & 1 for k in keys[lo[R[i]]:hi[i]]]
                assert set(left_bits) == {0} and set(right_bits) == {1}
            else:
                bit = (int(lo[i]) ^ int(hi[i] - 1)).bit_length() - 1
                assert all(((p >> bit) & 1) == 0 for p in range(lo[i], hi[L[i]]))
                assert all(((p >> bit) & 1) == 1 for p in range(lo[R[i]], hi[i]))
        sl = slice(lo[i], hi[i])
        M = ms[sl].sum()
        assert nd["mass"][i] == pytest.approx(M, rel=1e-14)
        com = (ms[sl, None] * xs[sl]).sum(0) / M
        assert nd["s"][i] == pytest.approx(com, rel=1e-12, abs=1e-14)
        dist = np.linalg.norm(xs[sl] - nd["s"][i], axis=1).max()
        assert nd["l"][i] == pytest.approx(dist, rel=1e-14, abs=1e-300)
        assert nd["hmax"][i] == hs[sl].max()
    leaves = t.leaves()
    assert np.all(L[leaves] < 0)
    assert np.all(np.diff(lo[leaves]) > 0)
    assert (hi[leaves] - lo[leaves]).sum() == n
    return t


@pytest.mark.parametrize("leaf_size", [1, 4, 10])
def test_tree_structure_plummer(orc, leaf_size):
    x, m, h = workloads.plummer(700, seed=3)
    _check_tree(orc, x, m, h, leaf_size)


def test_tree_with_duplicates(orc):
    rng = np.random.default_rng(1)
    base = rng.uniform(size=(40, 3))
    x = np.concatenate([base, base, base[:13], np.zeros((9, 3))])
    n = len(x)
    _check_tree(orc, x, rng.uniform(0.5, 1.5, n), rng.uniform(0.01, 0.1, n), 3)


def test_single_leaf_root(orc):
    x, m, h = workloads.plummer(10, seed=4)
    t = orc.Tree(x, m, h, leaf_size=10)
    assert t.num_nodes == 1 and t.num_leaves == 1


def test_moments_closed_form(orc):
    # 8 equal masses on the corners of a cube of half-side c about the origin:
    # odd moments vanish, Q~_(2,0,0) = M c^2 / 2, Q~_(1,1,0) = 0, Q~_(2,2,0)... etc.
    c = 0.3
    x = np.array([[sx * c, sy * c, sz * c] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)])
    m = np.full(8, 0.25)
    t = orc.Tree(x, m, np.ones(8), leaf_size=8, order=4)
    Q = t.moments()[0]
    M = m.sum()
    for k, (a, b, cc) in enumerate(orc.multi_indices(4)):
        if a % 2 or b % 2 or cc % 2:
            expect = 0.0
        else:
            expect = M * c ** (a + b + cc) / (math.factorial(a) * math.factorial(b)
                                              * math.factorial(cc))
        assert Q[k] == pytest.approx(expect, abs=1e-15)


def test_moments_translate_to_parent(orc):
    """Eq. (massmomtrans): the parent's moments are the children's moments
    re-centred by g = s_child - s_parent (binomial expansion of (g+b)^alpha)."""
    x, m, h = workloads.plummer(300, seed=8)
    t = orc.Tree(x, m, h, leaf_size=8, order=4)
    nd = t.nodes(); Q = t.moments(); mi = orc.multi_indices(4)
    idx = {tuple(a): k for k, a in enumerate(mi)}
    fac = lambda a: math.factorial(a[0]) * math.factorial(a[1]) * math.factorial(a[2])
    for i in range(t.num_nodes):
        if nd["left"][i] < 0:
            continue
        acc = np.zeros(len(mi))
        for ch in (nd["left"][i], nd["right"][i]):
            g = nd["s"][ch] - nd["s"][i]
            for k, a in enumerate(mi):
                for kb, b in enumerate(mi):
                    dlt = a - b
                    if np.any(dlt < 0):
                        continue
                    acc[k] += Q[ch, kb] * np.prod(g ** dlt) / fac(dlt)
        scale = np.abs(Q[i]).max()
        assert np.abs(acc - Q[i]).max() < 1e-13 * scale
