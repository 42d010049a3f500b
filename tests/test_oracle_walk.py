"""Pins of the oracle's interaction set (Algorithms 1 and 2, Sect. 3).

* every ordered particle pair (i, j) is covered exactly once, either by one
  M2L of an ancestor of i's leaf with a node holding j, or by one P2P leaf
  pair (brute-force count);
* the per-leaf lists are the recursive mutual traversal's pairs restricted to
  the leaf's branch, and that pair set is symmetric (Newton's third law);
* every accepted pair passes both criteria and keeps all of its particle
  pairs outside both softening kernels.
"""
import numpy as np
import pytest

import workloads


def _setup(orc, n=1500, seed=21, leaf_size=8, theta=0.6):
    x, m, h = workloads.plummer(n, seed=seed)
    t = orc.Tree(x, m, h, leaf_size=leaf_size, order=3)
    return t, x, m, h, theta


def _ancestors(nd, leaf):
    parent = {}
    for i in range(len(nd["lo"])):
        if nd["left"][i] >= 0:
            parent[nd["left"][i]] = i; parent[nd["right"][i]] = i
    br = [leaf]
    while br[-1] in parent:
        br.append(parent[br[-1]])
    return br[::-1]


@pytest.mark.parametrize("theta,r_kern", [(0.6, 2.0), (0.3, 2.0), (0.9, 0.0)])
def test_pair_partition(orc, theta, r_kern):
    t, x, m, h, _ = _setup(orc)
    nd = t.nodes(); n = t.n
    lo, hi = nd["lo"], nd["hi"]
    for leaf in t.leaves():
        dep, src, p2p = t.leaf_lists(leaf, theta, r_kern)
        cover = np.zeros(n, np.int32)
        br = _ancestors(nd, leaf)
        assert np.all(dep < len(br))
        for d, s in zip(dep, src):
            cover[lo[s]:hi[s]] += 1
            # the target ancestor at this depth never contains the source
            T = br[d]
            assert hi[s] <= lo[T] or lo[s] >= hi[T]
        for s in p2p:
            assert nd["left"][s] < 0
            cover[lo[s]:hi[s]] += 1
        assert np.all(cover == 1), (leaf, np.bincount(cover))
        assert leaf in set(p2p.tolist())


def test_per_leaf_equals_mutual_restricted(orc):
    t, x, m, h, theta = _setup(orc)
    nd = t.nodes()
    mt, ms, pa, pb = t.mutual_pairs(theta)
    m2l = set(zip(mt.tolist(), ms.tolist()))
    assert m2l == {(b, a) for a, b in m2l}          # symmetric M2L set
    p2p = set(zip(pa.tolist(), pb.tolist()))
    assert p2p == {(b, a) for a, b in p2p}
    assert len(m2l) == len(mt) and len(p2p) == len(pa)
    by_t = {}
    for a, b in m2l:
        by_t.setdefault(a, set()).add(b)
    for leaf in t.leaves()[::7]:
        dep, src, p2pl = t.leaf_lists(leaf, theta)
        br = _ancestors(nd, leaf)
        got = set(zip([br[d] for d in dep], src.tolist()))
        assert len(got) == len(src)
        want = {(a, b) for a in br for b in by_t.get(a, ())}
        assert got == want
        assert set(p2pl.tolist()) == {b for a, b in p2p if a == leaf}


def test_accepted_pairs_are_outside_kernels(orc):
    t, x, m, h, theta = _setup(orc, n=900, seed=5, theta=0.7)
    nd = t.nodes(); perm = t.perm()
    xs, hs = x[perm], h[perm]
    mt, ms, _, _ = t.mutual_pairs(theta)
    for a, b in zip(mt[::5], ms[::5]):
        d = np.linalg.norm(nd["s"][b] - nd["s"][a])
        assert nd["l"][a] + nd["l"][b] < theta * d
        assert d >= nd["l"][a] + nd["l"][b] + 2.0 * max(nd["hmax"][a], nd["hmax"][b])
        xa, xb = xs[nd["lo"][a]:nd["hi"][a]], xs[nd["lo"][b]:nd["hi"][b]]
        r = np.linalg.norm(xa[:, None, :] - xb[None, :, :], axis=2)
        hmax = np.maximum(hs[nd["lo"][a]:nd["hi"][a], None], hs[None, nd["lo"][b]:nd["hi"][b]])
        assert np.all(r >= 2.0 * hmax)


def test_secondary_criterion_forces_p2p(orc):
    """With R_kern h larger than the system every pair is opened down to P2P."""
    x, m, h = workloads.plummer(300, seed=6)
    t = orc.Tree(x, m, np.full(300, 1e3), leaf_size=8)
    mt, ms, pa, pb = t.mutual_pairs(0.9)
    assert len(mt) == 0
    assert len(pa) == t.num_leaves ** 2
