"""Seeded synthetic particle sets for the SFMM gravity solve.

Input generation only: this module holds none of the solver's arithmetic and
is shared by the tests, the benchmark and the smoke check, which feed the same
arrays to the HIP path and to the CPU oracle.  Every generator takes an
explicit seed and uses numpy's PCG64.

Recipes (stand-ins for the paper's initial conditions, which are not public):
  * plummer            -- Plummer sphere (Results, "Plummer and homogeneous
                          sphere"), equal masses, inverse-CDF radii; softening
                          from the analytic density, h = 1.2 (m/rho)^(1/3).
  * homogeneous_sphere -- uniform ball, same softening rule.
  * polytrope          -- n = 1.5 Lane-Emden sphere (the binary-polytrope test
                          uses gamma = 5/3 stars); softening lengths are half
                          the distance to the 58th nearest neighbour.
  * binary_polytrope   -- two such stars separated by 3 R.
  * lognormal_cloud    -- clumpy cloud from a log-normal random field.
  * serving_stream     -- a Poisson stream of independent small systems.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

NNGB = 58  # neighbours inside 2h: (4 pi / 3) (2 * 1.2)^3 ~ 58


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _isotropic(rng: np.random.Generator, r: np.ndarray) -> np.ndarray:
    n = len(r)
    mu = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return np.stack([r * s * np.cos(phi), r * s * np.sin(phi), r * mu], axis=1)


def h_from_neighbours(x: np.ndarray, k: int = NNGB, workers: int = -1) -> np.ndarray:
    """Half the distance to the k-th nearest other particle."""
    from scipy.spatial import cKDTree

    tree = cKDTree(x)
    d, _ = tree.query(x, k=k + 1, workers=workers)
    return 0.5 * d[:, k]


def plummer(n: int, seed: int = 1, a: float = 1.0, M: float = 1.0, rmax: float = 100.0):
    """Plummer sphere rho = 3 M a^2 / (4 pi (a^2 + r^2)^(5/2)) (the exponent's sign is
    garbled in the paper's text; this is the standard profile)."""
    rng = _rng(seed)
    r = np.empty(0)
    while len(r) < n:
        X = rng.uniform(0.0, 1.0, 2 * (n - len(r)) + 16)
        X = X[X > 0.0]
        rr = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        r = np.concatenate([r, rr[rr <= rmax * a]])
    r = r[:n]
    x = _isotropic(rng, r)
    m = np.full(n, M / n)
    rho = 3.0 * M / (4.0 * math.pi * a ** 3) * (1.0 + (r / a) ** 2) ** (-2.5)
    h = 1.2 * (m / rho) ** (1.0 / 3.0)
    return x, m, h


def homogeneous_sphere(n: int, seed: int = 11, R: float = 1.0, M: float = 1.0):
    rng = _rng(seed)
    r = R * rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    x = _isotropic(rng, r)
    m = np.full(n, M / n)
    rho = 3.0 * M / (4.0 * math.pi * R ** 3)
    h = np.full(n, 1.2 * (M / n / rho) ** (1.0 / 3.0))
    return x, m, h


def lane_emden(n_index: float = 1.5, dxi: float = 1e-4):
    """RK4 integration of theta'' + 2 theta'/xi + theta^n = 0 up to the first zero.

    Returns (xi, theta, dtheta) tables and xi_1 (the first zero, linearly
    interpolated)."""
    def rhs(xi, y):
        th, dth = y
        return np.array([dth, -max(th, 0.0) ** n_index - 2.0 * dth / xi])

    xi = 1e-6
    y = np.array([1.0 - xi * xi / 6.0, -xi / 3.0])
    xs, ths, dths = [0.0], [1.0], [0.0]
    while y[0] > 0.0:
        k1 = rhs(xi, y)
        k2 = rhs(xi + 0.5 * dxi, y + 0.5 * dxi * k1)
        k3 = rhs(xi + 0.5 * dxi, y + 0.5 * dxi * k2)
        k4 = rhs(xi + dxi, y + dxi * k3)
        y_new = y + dxi / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        if y_new[0] <= 0.0:
            frac = y[0] / (y[0] - y_new[0])
            xi1 = xi + frac * dxi
            xs.append(xi1); ths.append(0.0); dths.append(y[1] + frac * (y_new[1] - y[1]))
            break
        xi += dxi
        y = y_new
        xs.append(xi); ths.append(y[0]); dths.append(y[1])
    return np.array(xs), np.array(ths), np.array(dths), xs[-1]


_LE_CACHE: dict = {}


def _le_table(n_index: float):
    if n_index not in _LE_CACHE:
        _LE_CACHE[n_index] = lane_emden(n_index)
    return _LE_CACHE[n_index]


def polytrope_radii(rng: np.random.Generator, n: int, R: float = 1.0, n_index: float = 1.5):
    xi, th, dth, xi1 = _le_table(n_index)
    mass = -xi * xi * dth  # enclosed mass profile (arbitrary units)
    mass[0] = 0.0
    mass = np.maximum.accumulate(mass)
    u = rng.uniform(0.0, mass[-1], n)
    return R * np.interp(u, mass, xi) / xi1


def polytrope(n: int, seed: int = 2, R: float = 1.0, M: float = 1.0, center=(0.0, 0.0, 0.0),
              with_h: bool = True):
    rng = _rng(seed)
    r = polytrope_radii(rng, n, R)
    x = _isotropic(rng, r) + np.asarray(center, dtype=np.float64)
    m = np.full(n, M / n)
    h = h_from_neighbours(x) if with_h else None
    return x, m, h


def binary_polytrope(n_each: int, seeds=(3, 4), R: float = 1.0, M: float = 1.0):
    """Two n=1.5 stars of mass M at (+-1.5R, 0, 0); circular velocities
    (0, +-sqrt(G 2M / (3R)) / 2, 0) are returned for completeness."""
    xa, ma, _ = polytrope(n_each, seeds[0], R, M, (-1.5 * R, 0.0, 0.0), with_h=False)
    xb, mb, _ = polytrope(n_each, seeds[1], R, M, (1.5 * R, 0.0, 0.0), with_h=False)
    x = np.concatenate([xa, xb]); m = np.concatenate([ma, mb])
    h = h_from_neighbours(x)
    vc = 0.5 * math.sqrt(2.0 * M / (3.0 * R))
    v = np.zeros_like(x)
    v[:n_each, 1] = -vc; v[n_each:, 1] = vc
    return x, m, h, v


def lognormal_cloud(n: int, seed_field: int = 5, seed_particles: int = 6, grid: int = 128,
                    sigma_ln: float = 2.0, slope: float = -4.0):
    """Particles sampled from rho ~ exp(delta - sigma^2/2), delta a Gaussian field on a
    grid^3 mesh with power spectrum k^slope scaled to standard deviation sigma_ln."""
    rng = _rng(seed_field)
    k = np.fft.fftfreq(grid) * grid
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.zeros_like(kk)
    amp[kk > 0] = kk[kk > 0] ** (slope / 2.0)
    noise = rng.normal(size=(grid, grid, grid)) + 1j * rng.normal(size=(grid, grid, grid))
    field = np.real(np.fft.ifftn(noise * amp))
    field = (field - field.mean()) / field.std() * sigma_ln
    rho = np.exp(field - 0.5 * sigma_ln ** 2).ravel()
    p = rho / rho.sum()
    rng2 = _rng(seed_particles)
    cells = rng2.choice(len(p), size=n, p=p)
    ix, iy, iz = np.unravel_index(cells, (grid, grid, grid))
    x = (np.stack([ix, iy, iz], axis=1) + rng2.uniform(0.0, 1.0, (n, 3))) / grid
    m = np.full(n, 1.0 / n)
    h = h_from_neighbours(x)
    return x, m, h


@dataclass
class Request:
    rid: int
    arrival: float
    kind: str
    x: np.ndarray
    m: np.ndarray
    h: np.ndarray


def serving_stream(count: int = 512, seed: int = 7, rate: float = 200.0, nmin: float = 1e3,
                   nmax: float = 1e6, max_total: float | None = None):
    """Poisson arrivals of independent Plummer / polytrope systems with
    log-uniform N, scale and mass; softening from the analytic density."""
    rng = _rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(10 ** rng.uniform(math.log10(nmin), math.log10(nmax)))
        scale = 10 ** rng.uniform(math.log10(0.5), math.log10(2.0))
        M = 10 ** rng.uniform(math.log10(0.5), math.log10(2.0))
        sub = int(rng.integers(0, 2 ** 31))
        if i % 2 == 0:
            x, m, h = plummer(n, sub, a=scale, M=M)
            kind = "plummer"
        else:
            r = _rng(sub)
            rr = polytrope_radii(r, n, scale)
            x = _isotropic(r, rr)
            m = np.full(n, M / n)
            xi, th, dth, xi1 = _le_table(1.5)
            # analytic density of the n=1.5 polytrope at each radius
            rho_c = M / (4.0 * math.pi * (scale / xi1) ** 3 * (-xi1 ** 2 * dth[-1]))
            thr = np.interp(rr / scale * xi1, xi, th)
            rho = rho_c * np.maximum(thr, 1e-3) ** 1.5
            h = 1.2 * (m / rho) ** (1.0 / 3.0)
            kind = "polytrope"
        out.append(Request(i, t, kind, x, m, h))
        if max_total is not None and sum(len(q.m) for q in out) > max_total:
            break
    return out
