"""ctypes wrapper of the serial FP64 SFMM oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline leg of the benchmark are its only users.  The product library never
imports this package and this package never imports the product; they share
no code.  What each oracle function computes, and the passage of the paper it
follows, is documented in ``sfmm_oracle.h`` / ``sfmm_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sfmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# -ffp-contract=off: every operation rounds as written (no fused multiply-add),
# which the bit-exact tree/geometry comparisons rely on.
# -fopenmp: only orc_solve_parallel uses threads (each over whole leaves).
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared",
          "-fopenmp", "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (always recompiles)."""
    cmd = ["gcc", *CFLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        d, i32, i64, u64, vp = C.c_double, C.c_int32, C.c_int64, C.c_uint64, C.c_void_p
        L.orc_psi_hat.restype = d; L.orc_psi_hat.argtypes = [d]
        L.orc_f_hat.restype = d; L.orc_f_hat.argtypes = [d]
        L.orc_g.restype = d; L.orc_g.argtypes = [d, d]
        L.orc_psi.restype = d; L.orc_psi.argtypes = [d, d]
        L.orc_ncoef.restype = C.c_int; L.orc_ncoef.argtypes = [C.c_int]
        L.orc_multi_index.restype = C.c_int; L.orc_multi_index.argtypes = [C.c_int, vp]
        L.orc_derivs.restype = C.c_int; L.orc_derivs.argtypes = [C.c_int, vp, vp]
        L.orc_direct.restype = C.c_int
        L.orc_direct.argtypes = [i64, vp, vp, vp, d, C.c_int, vp, vp]
        L.orc_direct_targets.restype = C.c_int
        L.orc_direct_targets.argtypes = [i64, vp, vp, vp, d, C.c_int, i64, vp, vp, vp]
        L.orc_tree_build.restype = vp
        L.orc_tree_build.argtypes = [i64, vp, vp, vp, C.c_int, C.c_int]
        L.orc_tree_free.restype = None; L.orc_tree_free.argtypes = [vp]
        L.orc_tree_num_nodes.restype = i64; L.orc_tree_num_nodes.argtypes = [vp]
        L.orc_tree_num_leaves.restype = i64; L.orc_tree_num_leaves.argtypes = [vp]
        L.orc_tree_max_depth.restype = C.c_int; L.orc_tree_max_depth.argtypes = [vp]
        L.orc_tree_order.restype = C.c_int; L.orc_tree_order.argtypes = [vp]
        L.orc_tree_get_perm.restype = None; L.orc_tree_get_perm.argtypes = [vp, vp]
        L.orc_tree_get_keys.restype = None; L.orc_tree_get_keys.argtypes = [vp, vp]
        L.orc_tree_get_nodes.restype = None
        L.orc_tree_get_nodes.argtypes = [vp] * 10
        L.orc_tree_get_moments.restype = None; L.orc_tree_get_moments.argtypes = [vp, vp]
        L.orc_tree_get_leaves.restype = None; L.orc_tree_get_leaves.argtypes = [vp, vp]
        L.orc_leaf_lists.restype = i64
        L.orc_leaf_lists.argtypes = [vp, i32, d, d, vp, vp, i64, vp, i64, vp]
        L.orc_mutual_pairs.restype = i64
        L.orc_mutual_pairs.argtypes = [vp, d, d, vp, vp, i64, vp, vp, i64, vp]
        L.orc_solve.restype = C.c_int
        L.orc_solve.argtypes = [vp, d, d, d, C.c_int, C.c_int, i64, vp, vp, vp, vp]
        L.orc_solve_parallel.restype = C.c_int
        L.orc_solve_parallel.argtypes = [vp, d, d, d, C.c_int, C.c_int, vp, vp, vp, vp]
        L.orc_sfmm_solve.restype = C.c_int
        L.orc_sfmm_solve.argtypes = [i64, vp, vp, vp, d, C.c_int, C.c_int, d, d, C.c_int,
                                     vp, vp, vp]
        L.orc_m2l_pair.restype = C.c_int
        L.orc_m2l_pair.argtypes = [C.c_int, i64, vp, vp, vp, i64, vp, vp, d, vp, vp]
        _ = (u64,)
        _lib = L
    return _lib


class Stats(C.Structure):
    _fields_ = [("n_m2l", C.c_int64), ("n_p2p_pairs", C.c_int64),
                ("n_leaves_done", C.c_int64)]


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# ---- kernel and derivative helpers ----------------------------------------
def psi_hat(q: float) -> float:
    return lib().orc_psi_hat(float(q))


def f_hat(q: float) -> float:
    return lib().orc_f_hat(float(q))


def g(r: float, h: float) -> float:
    return lib().orc_g(float(r), float(h))


def psi(r: float, h: float) -> float:
    return lib().orc_psi(float(r), float(h))


def ncoef(order: int) -> int:
    return lib().orc_ncoef(order)


def multi_indices(order: int) -> np.ndarray:
    out = np.zeros((ncoef(order), 3), dtype=np.int32)
    buf = np.zeros(3, dtype=np.int32)
    for k in range(ncoef(order)):
        lib().orc_multi_index(k, _p(buf))
        out[k] = buf
    return out


def derivs(order: int, r) -> np.ndarray:
    r = _f64(r, (3,))
    out = np.zeros(ncoef(order))
    if lib().orc_derivs(order, _p(r), _p(out)) != 0:
        raise ValueError("orc_derivs failed")
    return out


# ---- direct sum -------------------------------------------------------------
def direct(x, m, h, G=1.0, include_self=True, targets=None):
    x = _f64(x, (-1, 3)); m = _f64(m); h = _f64(h)
    n = len(m)
    if targets is None:
        acc = np.zeros((n, 3)); pot = np.zeros(n)
        rc = lib().orc_direct(n, _p(x), _p(m), _p(h), G, int(include_self), _p(acc), _p(pot))
    else:
        t = np.ascontiguousarray(targets, dtype=np.int64)
        acc = np.zeros((len(t), 3)); pot = np.zeros(len(t))
        rc = lib().orc_direct_targets(n, _p(x), _p(m), _p(h), G, int(include_self), len(t),
                                      _p(t), _p(acc), _p(pot))
    if rc != 0:
        raise ValueError("orc_direct failed")
    return acc, pot


# ---- tree + solve -------------------------------------------------------------
MODE_PER_LEAF, MODE_MUTUAL, MODE_DIRECT_ANC = 0, 1, 2


class Tree:
    """Oracle tree over (x, m, h): Morton keys, binary radix split, geometry, moments."""

    def __init__(self, x, m, h, leaf_size=10, order=3):
        self.x = _f64(x, (-1, 3)); self.m = _f64(m); self.h = _f64(h)
        self.n = len(self.m)
        self.order = order
        self._t = lib().orc_tree_build(self.n, _p(self.x), _p(self.m), _p(self.h),
                                       leaf_size, order)
        if not self._t:
            raise ValueError("orc_tree_build failed")

    def __del__(self):
        if getattr(self, "_t", None):
            lib().orc_tree_free(self._t)
            self._t = None

    @property
    def num_nodes(self):
        return lib().orc_tree_num_nodes(self._t)

    @property
    def num_leaves(self):
        return lib().orc_tree_num_leaves(self._t)

    @property
    def max_depth(self):
        return lib().orc_tree_max_depth(self._t)

    def perm(self):
        out = np.zeros(self.n, dtype=np.int64)
        lib().orc_tree_get_perm(self._t, _p(out))
        return out

    def keys(self):
        out = np.zeros(self.n, dtype=np.uint64)
        lib().orc_tree_get_keys(self._t, _p(out))
        return out

    def nodes(self):
        nn = self.num_nodes
        d = dict(lo=np.zeros(nn, np.int64), hi=np.zeros(nn, np.int64),
                 left=np.zeros(nn, np.int32), right=np.zeros(nn, np.int32),
                 depth=np.zeros(nn, np.int32), s=np.zeros((nn, 3)), mass=np.zeros(nn),
                 l=np.zeros(nn), hmax=np.zeros(nn))
        lib().orc_tree_get_nodes(self._t, *[_p(d[k]) for k in
                                            ("lo", "hi", "left", "right", "depth", "s", "mass",
                                             "l", "hmax")])
        return d

    def moments(self):
        out = np.zeros((self.num_nodes, ncoef(self.order)))
        lib().orc_tree_get_moments(self._t, _p(out))
        return out

    def leaves(self):
        out = np.zeros(self.num_leaves, dtype=np.int32)
        lib().orc_tree_get_leaves(self._t, _p(out))
        return out

    def leaf_lists(self, leaf, theta, r_kern=2.0):
        np2p = C.c_int64(0)
        n = lib().orc_leaf_lists(self._t, int(leaf), theta, r_kern, None, None, 0, None, 0,
                                 C.byref(np2p))
        if n < 0:
            raise ValueError("not a leaf")
        dep = np.zeros(n, np.int32); src = np.zeros(n, np.int32)
        p2p = np.zeros(np2p.value, np.int32)
        lib().orc_leaf_lists(self._t, int(leaf), theta, r_kern, _p(dep), _p(src), n, _p(p2p),
                             len(p2p), C.byref(np2p))
        return dep, src, p2p

    def mutual_pairs(self, theta, r_kern=2.0):
        np2p = C.c_int64(0)
        n = lib().orc_mutual_pairs(self._t, theta, r_kern, None, None, 0, None, None, 0,
                                   C.byref(np2p))
        mt = np.zeros(n, np.int32); ms = np.zeros(n, np.int32)
        pa = np.zeros(np2p.value, np.int32); pb = np.zeros(np2p.value, np.int32)
        lib().orc_mutual_pairs(self._t, theta, r_kern, _p(mt), _p(ms), n, _p(pa), _p(pb),
                               len(pa), C.byref(np2p))
        return mt, ms, pa, pb

    def solve(self, theta=0.5, G=1.0, r_kern=2.0, include_self=True, mode=MODE_PER_LEAF,
              targets=None):
        st = Stats()
        if targets is None:
            acc = np.zeros((self.n, 3)); pot = np.zeros(self.n)
            rc = lib().orc_solve(self._t, theta, G, r_kern, int(include_self), mode, -1, None,
                                 _p(acc), _p(pot), C.byref(st))
        else:
            t = np.ascontiguousarray(targets, dtype=np.int64)
            acc = np.zeros((len(t), 3)); pot = np.zeros(len(t))
            rc = lib().orc_solve(self._t, theta, G, r_kern, int(include_self), mode, len(t),
                                 _p(t), _p(acc), _p(pot), C.byref(st))
        if rc != 0:
            raise ValueError("orc_solve failed")
        return acc, pot, dict(n_m2l=st.n_m2l, n_p2p_pairs=st.n_p2p_pairs,
                              n_leaves_done=st.n_leaves_done)

    def solve_parallel(self, theta=0.5, G=1.0, r_kern=2.0, include_self=True, nthreads=0):
        """Algorithm 1 with the loop over leaves on OpenMP threads (every
        particle); equal to solve() bit for bit.  Also returns the threads used."""
        st = Stats()
        used = C.c_int(0)
        acc = np.zeros((self.n, 3)); pot = np.zeros(self.n)
        rc = lib().orc_solve_parallel(self._t, theta, G, r_kern, int(include_self), int(nthreads),
                                      _p(acc), _p(pot), C.byref(st), C.byref(used))
        if rc != 0:
            raise ValueError("orc_solve_parallel failed")
        return acc, pot, dict(n_m2l=st.n_m2l, n_p2p_pairs=st.n_p2p_pairs,
                              n_leaves_done=st.n_leaves_done, threads=used.value)


def sfmm_solve(x, m, h, theta=0.5, order=3, leaf_size=10, G=1.0, r_kern=2.0,
               include_self=True):
    x = _f64(x, (-1, 3)); m = _f64(m); h = _f64(h)
    n = len(m)
    acc = np.zeros((n, 3)); pot = np.zeros(n)
    st = Stats()
    rc = lib().orc_sfmm_solve(n, _p(x), _p(m), _p(h), theta, order, leaf_size, G, r_kern,
                              int(include_self), _p(acc), _p(pot), C.byref(st))
    if rc != 0:
        raise ValueError("orc_sfmm_solve failed")
    return acc, pot


def m2l_pair(order, xs, ms, sS, xt, sT, G=1.0):
    xs = _f64(xs, (-1, 3)); ms = _f64(ms); xt = _f64(xt, (-1, 3))
    sS = _f64(sS, (3,)); sT = _f64(sT, (3,))
    acc = np.zeros((len(xt), 3)); pot = np.zeros(len(xt))
    rc = lib().orc_m2l_pair(order, len(ms), _p(xs), _p(ms), _p(sS), len(xt), _p(xt), _p(sT),
                            G, _p(acc), _p(pot))
    if rc != 0:
        raise ValueError("orc_m2l_pair failed")
    return acc, pot
