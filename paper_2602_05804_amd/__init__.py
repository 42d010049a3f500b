"""MI355X (gfx950) SFMM gravity solve: Python binding of libsfmm.so.

Symmetric Cartesian fast multipole method with adaptive cubic-spline
softening (Bernard et al., arXiv 2602.05804): Morton radix tree, the per-leaf
dual tree walk of Algorithms 1-2, M2L / L2L / L2P expansions and softened
P2P, all in hand-written HIP kernels behind the C ABI of ``include/sfmm.h``.

This module only marshals arguments: torch supplies device memory and the
current HIP stream, every step of the solve runs in libsfmm.so.  There is no
CPU fallback: if the library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

__all__ = ["Solver", "SfmmError", "solve", "lib", "LIB_PATH", "EXPORTED", "FLOPS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfmm.so")

# every entry point declared in include/sfmm.h
EXPORTED = ("sfmm_config_default", "sfmm_create", "sfmm_destroy", "sfmm_set_stream",
            "sfmm_build", "sfmm_solve", "sfmm_solve_batch", "sfmm_get_stats", "sfmm_get_tree", "sfmm_get_leaves",
            "sfmm_get_leaf_lists", "sfmm_timing_start", "sfmm_timing_stop", "sfmm_phase_name",
            "sfmm_workspace_bytes", "sfmm_leapfrog", "sfmm_direct", "sfmm_direct_noalloc",
            "sfmm_strerror", "sfmm_last_error")
PHASES = ("tree", "walk_count", "walk_fill", "far", "near", "momentum", "near_kernel")

# floating-point operations per unit of work at each expansion order, counted
# from the generated kernels (FMA = 2); see csrc/expansions_gen.h
FLOPS = {
    "m2l": {0: 24, 1: 97, 2: 280, 3: 659, 4: 1362},
    # one unordered pair in both directions (the mutual far field)
    "m2l_pair": {0: 32, 1: 144, 2: 437, 3: 1068, 4: 2278},
    "l2l": {0: 0, 1: 27, 2: 138, 3: 438, 4: 1105},
    "l2p": {0: 4, 1: 31, 2: 88, 3: 184, 4: 329},
}

SFMM_FP64, SFMM_FP32C = 0, 1
_PRECISION = {"fp64": SFMM_FP64, "fp32c": SFMM_FP32C}


class SfmmError(RuntimeError):
    """A failed call; `code` is the sfmm_status value (0 when the error was
    found in Python, before any call)."""

    def __init__(self, msg, code: int = 0):
        super().__init__(msg)
        self.code = int(code)


# sfmm_status values
SFMM_EINVAL, SFMM_ENOMEM, SFMM_EDEVICE, SFMM_EUNSUPPORTED, SFMM_ENONFINITE = -1, -2, -3, -4, -5


class Config(C.Structure):
    _fields_ = [("G", C.c_double), ("leaf_size", C.c_int), ("r_kern", C.c_double),
                ("include_self_potential", C.c_int), ("check_inputs", C.c_int),
                ("walk_mode", C.c_int), ("fp64_top_depth", C.c_int), ("far_mode", C.c_int),
                ("far_kernel", C.c_int), ("near_kernel", C.c_int)]


WALK_MODES = {"level": 0, "leaf": 1}
FAR_MODES = {"leaf": 0, "shared": 1, "mutual": 2}


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("num_nodes", C.c_int64), ("num_leaves", C.c_int64),
                ("max_depth", C.c_int32), ("n_m2l", C.c_int64), ("n_l2l", C.c_int64),
                ("n_p2p_leaf_pairs", C.c_int64), ("n_p2p_pairs", C.c_int64),
                ("momentum", C.c_double * 3), ("momentum_abs", C.c_double),
                ("n_m2l_unique", C.c_int64), ("n_p2p_soft_pairs", C.c_int64),
                ("walk_attempts", C.c_int32), ("leaf_slot_m2l", C.c_int32),
                ("leaf_slot_p2p", C.c_int32), ("n_leaf_overflow", C.c_int64),
                ("max_leaf_m2l", C.c_int64), ("max_leaf_p2p", C.c_int64)]


_lib = None


def lib():
    """Load libsfmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SfmmError(f"{LIB_PATH} is missing: build it with "
                            "`python -m paper_2602_05804_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.sfmm_config_default.argtypes = [vp]
        L.sfmm_create.argtypes = [C.POINTER(vp), C.c_int, vp, vp]
        L.sfmm_destroy.argtypes = [vp]
        L.sfmm_set_stream.argtypes = [vp, vp]
        L.sfmm_build.argtypes = [vp, i64, vp, vp, vp, C.c_int]
        L.sfmm_solve.argtypes = [vp, i64, vp, vp, vp, d, C.c_int, C.c_int, vp, vp]
        L.sfmm_solve_batch.argtypes = [vp, C.c_int, vp, vp, vp, vp, d, C.c_int, C.c_int, vp, vp]
        L.sfmm_get_stats.argtypes = [vp, vp]
        L.sfmm_get_tree.argtypes = [vp] * 14
        L.sfmm_get_leaves.argtypes = [vp, vp, vp]
        L.sfmm_get_leaf_lists.argtypes = [vp, i64, vp, vp, i64, vp, vp, i64, vp]
        L.sfmm_timing_start.argtypes = [vp, C.c_int]
        L.sfmm_timing_stop.argtypes = [vp, vp, C.c_int, vp]
        L.sfmm_phase_name.restype = C.c_char_p
        L.sfmm_phase_name.argtypes = [C.c_int]
        L.sfmm_workspace_bytes.argtypes = [vp, vp]
        L.sfmm_leapfrog.argtypes = [vp, i64, vp, vp, vp, d, d]
        L.sfmm_direct.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp, vp]
        L.sfmm_direct_noalloc.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp, vp]
        L.sfmm_strerror.restype = C.c_char_p
        L.sfmm_strerror.argtypes = [C.c_int]
        L.sfmm_last_error.restype = C.c_char_p
        L.sfmm_last_error.argtypes = [vp]
        for name in EXPORTED:
            if name not in ("sfmm_strerror", "sfmm_last_error", "sfmm_phase_name"):
                getattr(L, name).restype = C.c_int
        _ = i32
        _lib = L
    return _lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


class Solver:
    """A libsfmm context on one device; keeps its workspace between solves."""

    def __init__(self, device: int = 0, G: float = 1.0, leaf_size: int = 10,
                 r_kern: float = 2.0, include_self_potential: bool = True,
                 check_inputs: bool = True, walk: str = "level", fp64_top_depth: int = 8,
                 far: str = "shared", far_kernel: int = 0, near_kernel: int = 0):
        import torch

        if not torch.cuda.is_available():
            raise SfmmError("no HIP device available: the SFMM solve runs only on the GPU")
        self._torch = torch
        self.device = int(device)
        self.cfg = Config(G, leaf_size, r_kern, int(include_self_potential), int(check_inputs),
                          WALK_MODES[walk], int(fp64_top_depth), FAR_MODES[far],
                          int(far_kernel), int(near_kernel))
        self._ctx = C.c_void_p(0)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self._check(lib().sfmm_create(C.byref(self._ctx), self.device, C.c_void_p(stream),
                                      C.byref(self.cfg)), "sfmm_create")

    def _check(self, rc, what):
        if rc != 0:
            msg = lib().sfmm_strerror(rc).decode()
            extra = lib().sfmm_last_error(self._ctx).decode() if self._ctx else ""
            raise SfmmError(f"{what}: {msg} ({rc}) {extra}".strip(), rc)

    def _inputs(self, x, m, h):
        torch = self._torch
        dev = torch.device("cuda", self.device)
        for name, t in (("x", x), ("m", m), ("h", h)):
            if not isinstance(t, torch.Tensor):
                raise TypeError(f"{name} must be a torch tensor")
            if t.dtype != torch.float64:
                raise TypeError(f"{name} must be float64")
            if t.device != dev:
                raise ValueError(f"{name} must live on {dev}")
            if not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous")
        n = m.shape[0]
        if x.shape != (n, 3) or m.shape != (n,) or h.shape != (n,):
            raise ValueError("expected x [n,3], m [n], h [n]")
        lib().sfmm_set_stream(self._ctx, C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
        return n

    def build(self, x, m, h, order: int = 3):
        n = self._inputs(x, m, h)
        self._check(lib().sfmm_build(self._ctx, n, _ptr(x), _ptr(m), _ptr(h), order),
                    "sfmm_build")

    def solve(self, x, m, h, theta: float = 0.5, order: int = 3, precision: str = "fp64",
              acc=None, pot=None):
        """Accelerations [n,3] and potentials [n] (float64, device, caller order)."""
        torch = self._torch
        n = self._inputs(x, m, h)
        if precision not in _PRECISION:
            raise SfmmError(f"unknown precision {precision!r}")
        if acc is None:
            acc = torch.empty((n, 3), dtype=torch.float64, device=x.device)
        if pot is None:
            pot = torch.empty((n,), dtype=torch.float64, device=x.device)
        self._check(lib().sfmm_solve(self._ctx, n, _ptr(x), _ptr(m), _ptr(h), float(theta),
                                     int(order), _PRECISION[precision], _ptr(acc), _ptr(pot)),
                    "sfmm_solve")
        return acc, pot

    def solve_batch(self, systems, theta: float = 0.5, order: int = 3, precision: str = "fp64"):
        """Solve several independent systems in one pass; systems is a list of
        (x, m, h) device tensors.  Returns a list of (acc, pot), each exactly
        what a solve of that system alone returns."""
        import numpy as np

        torch = self._torch
        if len(systems) == 0:
            return []
        for i, (x, m, h) in enumerate(systems):
            if not (x.dim() == 2 and x.shape[1] == 3 and m.shape == (x.shape[0],)
                    and h.shape == (x.shape[0],)):
                raise SfmmError(f"system {i}: x must be [n, 3] and m, h [n]")
        xs = torch.cat([s[0] for s in systems]).contiguous()
        ms = torch.cat([s[1] for s in systems]).contiguous()
        hs = torch.cat([s[2] for s in systems]).contiguous()
        n = self._inputs(xs, ms, hs)
        if precision not in _PRECISION:
            raise SfmmError(f"unknown precision {precision!r}")
        off = np.zeros(len(systems) + 1, dtype=np.int64)
        off[1:] = np.cumsum([s[1].shape[0] for s in systems])
        acc = torch.empty((n, 3), dtype=torch.float64, device=xs.device)
        pot = torch.empty((n,), dtype=torch.float64, device=xs.device)
        self._check(lib().sfmm_solve_batch(self._ctx, len(systems), off.ctypes.data_as(C.c_void_p),
                                           _ptr(xs), _ptr(ms), _ptr(hs), float(theta), int(order),
                                           _PRECISION[precision], _ptr(acc), _ptr(pot)),
                    "sfmm_solve_batch")
        return [(acc[off[i]:off[i + 1]], pot[off[i]:off[i + 1]]) for i in range(len(systems))]

    def direct(self, x, m, h, targets=None, no_alloc=False, out=None):
        """Softened direct sum over all particles for `targets` (a device int64
        tensor of indices, or None for every particle): (acc [nt, 3], pot [nt]).
        no_alloc: through sfmm_direct_noalloc (the library allocates nothing;
        pass `out` = (acc, pot) to allocate nothing here either)."""
        torch = self._torch
        n = self._inputs(x, m, h)
        if targets is None:
            nt, tp = n, C.c_void_p(0)
        else:
            targets = targets.to(device=x.device, dtype=torch.int64).contiguous()
            nt, tp = int(targets.shape[0]), _ptr(targets)
        if out is None:
            acc = torch.empty((nt, 3), dtype=torch.float64, device=x.device)
            pot = torch.empty((nt,), dtype=torch.float64, device=x.device)
        else:
            acc, pot = out
            if tuple(acc.shape) != (nt, 3) or tuple(pot.shape) != (nt,) or \
                    acc.dtype != torch.float64 or pot.dtype != torch.float64 or \
                    not acc.is_contiguous() or not pot.is_contiguous():
                raise SfmmError("out must be contiguous float64 tensors [nt, 3] and [nt]")
        fn = lib().sfmm_direct_noalloc if no_alloc else lib().sfmm_direct
        name = "sfmm_direct_noalloc" if no_alloc else "sfmm_direct"
        self._check(fn(self._ctx, n, _ptr(x), _ptr(m), _ptr(h), nt, tp, _ptr(acc), _ptr(pot)),
                    name)
        return acc, pot

    def stats(self) -> dict:
        st = Stats()
        self._check(lib().sfmm_get_stats(self._ctx, C.byref(st)), "sfmm_get_stats")
        return dict(n=st.n, num_nodes=st.num_nodes, num_leaves=st.num_leaves,
                    max_depth=st.max_depth, n_m2l=st.n_m2l, n_l2l=st.n_l2l,
                    n_p2p_leaf_pairs=st.n_p2p_leaf_pairs, n_p2p_pairs=st.n_p2p_pairs,
                    momentum=list(st.momentum), momentum_abs=st.momentum_abs,
                    n_m2l_unique=st.n_m2l_unique, n_p2p_soft_pairs=st.n_p2p_soft_pairs,
                    walk_attempts=st.walk_attempts, leaf_slot_m2l=st.leaf_slot_m2l,
                    leaf_slot_p2p=st.leaf_slot_p2p, n_leaf_overflow=st.n_leaf_overflow,
                    max_leaf_m2l=st.max_leaf_m2l, max_leaf_p2p=st.max_leaf_p2p)

    def timing_start(self, max_solves: int):
        """Record HIP events around every phase of the next max_solves solves."""
        self._check(lib().sfmm_timing_start(self._ctx, int(max_solves)), "sfmm_timing_start")

    def timing_stop(self):
        """Phase durations (ms) of the recorded solves: list of dicts."""
        import numpy as np

        cap = 100000
        ns = C.c_int(0)
        # first call: learn how many were recorded without freeing the events
        buf = np.zeros((4096, len(PHASES)))
        self._check(lib().sfmm_timing_stop(self._ctx, buf.ctypes.data_as(C.c_void_p), 4096,
                                           C.byref(ns)), "sfmm_timing_stop")
        _ = cap
        return [dict(zip(PHASES, row)) for row in buf[:min(ns.value, 4096)]]

    def tree(self, order: int = 3) -> dict:
        import numpy as np

        nn, nl = C.c_int64(0), C.c_int64(0)
        self._check(lib().sfmm_get_tree(self._ctx, C.byref(nn), C.byref(nl), *([None] * 11)),
                    "sfmm_get_tree")
        st = self.stats()
        n, nn = st["n"], nn.value
        nq = (order + 1) * (order + 2) * (order + 3) // 6
        out = dict(perm=np.zeros(n, np.int32), keys=np.zeros(n, np.uint64),
                   lo=np.zeros(nn, np.int32), cnt=np.zeros(nn, np.int32),
                   child=np.zeros(nn, np.int32), parent=np.zeros(nn, np.int32),
                   s=np.zeros((nn, 3)), mass=np.zeros(nn), l=np.zeros(nn), hmax=np.zeros(nn),
                   Q=np.zeros((nn, nq)))
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        self._check(lib().sfmm_get_tree(self._ctx, None, None, *[p(out[k]) for k in (
            "perm", "keys", "lo", "cnt", "child", "parent", "s", "mass", "l", "hmax", "Q")]),
            "sfmm_get_tree")
        out["num_leaves"] = nl.value
        return out

    def leaves(self):
        import numpy as np

        nl = self.stats()["num_leaves"]
        node = np.zeros(nl, np.int32); depth = np.zeros(nl, np.int32)
        self._check(lib().sfmm_get_leaves(self._ctx, node.ctypes.data_as(C.c_void_p),
                                          depth.ctypes.data_as(C.c_void_p)), "sfmm_get_leaves")
        return node, depth

    def leaf_lists(self, leaf: int):
        import numpy as np

        nm, npp = C.c_int64(0), C.c_int64(0)
        self._check(lib().sfmm_get_leaf_lists(self._ctx, leaf, None, None, 0, C.byref(nm), None,
                                              0, C.byref(npp)), "sfmm_get_leaf_lists")
        dep = np.zeros(nm.value, np.int32); src = np.zeros(nm.value, np.int32)
        p2p = np.zeros(npp.value, np.int32)
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        self._check(lib().sfmm_get_leaf_lists(self._ctx, leaf, p(dep), p(src), nm.value,
                                              C.byref(nm), p(p2p), npp.value, C.byref(npp)),
                    "sfmm_get_leaf_lists")
        return dep, src, p2p

    def workspace_bytes(self) -> int:
        out = C.c_uint64(0)
        self._check(lib().sfmm_workspace_bytes(self._ctx, C.byref(out)), "sfmm_workspace_bytes")
        return out.value

    def close(self):
        if getattr(self, "_ctx", None):
            lib().sfmm_destroy(self._ctx)
            self._ctx = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def leapfrog(x, v, acc, kick: float, drift: float):
    """v += kick * acc; x += drift * v (device tensors [n,3], current stream)."""
    import torch

    rc = lib().sfmm_leapfrog(C.c_void_p(torch.cuda.current_stream(x.device).cuda_stream),
                             x.shape[0], _ptr(x), _ptr(v), _ptr(acc), float(kick), float(drift))
    if rc != 0:
        raise SfmmError(f"sfmm_leapfrog: {lib().sfmm_strerror(rc).decode()}")


_default: dict = {}


def solve(x, m, h, theta: float = 0.5, order: int = 3, precision: str = "fp64", **cfg):
    """One-call solve on x's device with a cached context per (device, config)."""
    key = (x.device.index or 0, tuple(sorted(cfg.items())))
    if key not in _default:
        _default[key] = Solver(device=key[0], **cfg)
    return _default[key].solve(x, m, h, theta=theta, order=order, precision=precision)
