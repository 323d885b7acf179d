"""Seeded synthetic particle sets for the RCB tree hot path.

This module only *makes inputs*: positions, masses, smoothing lengths and
cotangents. It holds none of the tree method's arithmetic, and both the CPU
oracle tests and the GPU path draw their inputs from it.

The paper benchmarks a Sobol sphere and two SPH snapshots (Sec. 3). The
snapshots are not available, so these clouds stand in for them: a uniform
sphere (the homogeneous case), a Plummer sphere, a Plummer sphere embedded in
a uniform background of 10% of the mass (a density contrast of ~1e4, like the
large smoothing-length range of the snapshots), and a unit cube with 64
Gaussian clumps. All masses are equal (1/N) and G = 1.

Smoothing lengths follow from the analytic number density n(r) so that about
50 neighbours fall inside the kernel support 2h:
    (4/3) pi (2h)^3 n = 50   =>   h = 0.5 * (150 / (4 pi n))^(1/3).
The small uniform sphere instead uses the exact k-nearest-neighbour distances
so that every particle has exactly 50 neighbours: h = (d50 + d51) / 4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 11080028
N_NEIGH = 50

PLUMMER_RMAX = 20.0
BG_RADIUS = 10.357          # uniform background radius, rho_P(0)/rho_bg ~ 1e4


@dataclass
class Cloud:
    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray
    h: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return self.x, self.y, self.z, self.m, self.h


def _isotropic(rng: np.random.Generator, r: np.ndarray):
    mu = rng.uniform(-1.0, 1.0, r.shape[0])
    phi = rng.uniform(0.0, 2.0 * math.pi, r.shape[0])
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return r * s * np.cos(phi), r * s * np.sin(phi), r * mu


def _h_from_density(n: np.ndarray, n_neigh: int = N_NEIGH) -> np.ndarray:
    return 0.5 * np.cbrt(3.0 * n_neigh / (4.0 * math.pi * n))


def plummer_mass(r):
    """Enclosed mass of a unit Plummer sphere (b = 1, M = 1)."""
    return r ** 3 / (1.0 + r * r) ** 1.5


def _plummer_radii(rng, n):
    xm = rng.uniform(0.0, plummer_mass(PLUMMER_RMAX), n)
    xm = np.maximum(xm, 1e-300)
    return 1.0 / np.sqrt(xm ** (-2.0 / 3.0) - 1.0)


def _plummer_number_density(r, n_p):
    rho = 3.0 / (4.0 * math.pi) * (1.0 + r * r) ** (-2.5)
    return n_p * rho / plummer_mass(PLUMMER_RMAX)


def knn_h(x, y, z, k: int = N_NEIGH, block: int = 1024) -> np.ndarray:
    """h = (d_k + d_{k+1}) / 4 from brute-force distances (self excluded)."""
    p = np.stack([x, y, z], axis=1)
    n = p.shape[0]
    h = np.empty(n)
    for s in range(0, n, block):
        q = p[s:s + block]
        d2 = ((q[:, None, :] - p[None, :, :]) ** 2).sum(-1)
        d2[np.arange(q.shape[0]), np.arange(s, s + q.shape[0])] = np.inf
        part = np.partition(d2, (k - 1, k), axis=1)
        h[s:s + block] = 0.25 * (np.sqrt(part[:, k - 1]) + np.sqrt(part[:, k]))
    return h


def uniform_sphere(n: int = 4096, seed: int = SEED_BASE + 1) -> Cloud:
    rng = np.random.default_rng(seed)
    r = np.cbrt(rng.uniform(0.0, 1.0, n))
    x, y, z = _isotropic(rng, r)
    m = np.full(n, 1.0 / n)
    return Cloud("uniform_sphere", x, y, z, m, knn_h(x, y, z))


def plummer(n: int = 1 << 20, seed: int = SEED_BASE + 2) -> Cloud:
    rng = np.random.default_rng(seed)
    r = _plummer_radii(rng, n)
    x, y, z = _isotropic(rng, r)
    m = np.full(n, 1.0 / n)
    h = _h_from_density(_plummer_number_density(r, n))
    return Cloud("plummer", x, y, z, m, h)


def plummer_background(n: int = 1 << 22, seed: int = SEED_BASE + 3,
                       bg_frac: float = 0.1) -> Cloud:
    rng = np.random.default_rng(seed)
    n_bg = int(round(bg_frac * n))
    n_p = n - n_bg
    rp = _plummer_radii(rng, n_p)
    rb = BG_RADIUS * np.cbrt(rng.uniform(0.0, 1.0, n_bg))
    r = np.concatenate([rp, rb])
    x, y, z = _isotropic(rng, r)
    perm = rng.permutation(n)            # interleave the two populations
    x, y, z, r = x[perm], y[perm], z[perm], r[perm]
    n_bg_dens = n_bg / (4.0 / 3.0 * math.pi * BG_RADIUS ** 3)
    dens = _plummer_number_density(r, n_p) + np.where(r <= BG_RADIUS, n_bg_dens, 0.0)
    m = np.full(n, 1.0 / n)
    return Cloud("plummer_background", x, y, z, m, _h_from_density(dens))


def clumpy_cube(n: int = 100_000_000, seed: int = SEED_BASE + 4,
                n_clumps: int = 64, sigma: float = 0.01) -> Cloud:
    rng = np.random.default_rng(seed)
    n_u = n // 2
    n_c = n - n_u
    per = np.full(n_clumps, n_c // n_clumps)
    per[: n_c % n_clumps] += 1
    centres = rng.uniform(0.1, 0.9, (n_clumps, 3))
    x = np.empty(n)
    y = np.empty(n)
    z = np.empty(n)
    x[:n_u] = rng.uniform(0.0, 1.0, n_u)
    y[:n_u] = rng.uniform(0.0, 1.0, n_u)
    z[:n_u] = rng.uniform(0.0, 1.0, n_u)
    s = n_u
    for c in range(n_clumps):
        k = int(per[c])
        x[s:s + k] = rng.normal(centres[c, 0], sigma, k)
        y[s:s + k] = rng.normal(centres[c, 1], sigma, k)
        z[s:s + k] = rng.normal(centres[c, 2], sigma, k)
        s += k
    perm = rng.permutation(n)
    x, y, z = x[perm], y[perm], z[perm]
    inside = (x >= 0) & (x <= 1) & (y >= 0) & (y <= 1) & (z >= 0) & (z <= 1)
    dens = np.where(inside, float(n_u), 0.0)
    norm = (2.0 * math.pi * sigma * sigma) ** -1.5
    cut = 8.0 * sigma
    # particles binned on a grid of cells no smaller than the cut, so each
    # clump only looks at the cells its cut box touches
    G = max(1, int(1.0 / cut))
    cell = lambda v: np.clip(np.floor(v * G), 0, G - 1).astype(np.int16)
    key = (cell(x) * G + cell(y)) * G + cell(z)
    order = np.argsort(key, kind="stable")
    bounds = np.searchsorted(key[order], np.arange(G ** 3 + 1))
    for c in range(n_clumps):
        cx, cy, cz = centres[c]
        lo = [int(np.clip(np.floor((v - cut) * G), 0, G - 1)) for v in (cx, cy, cz)]
        hi = [int(np.clip(np.floor((v + cut) * G), 0, G - 1)) for v in (cx, cy, cz)]
        cand = np.concatenate([order[bounds[(i * G + j) * G + lo[2]]:bounds[(i * G + j) * G + hi[2] + 1]]
                               for i in range(lo[0], hi[0] + 1) for j in range(lo[1], hi[1] + 1)])
        sel = cand[(np.abs(x[cand] - cx) < cut) & (np.abs(y[cand] - cy) < cut) & (np.abs(z[cand] - cz) < cut)]
        d2 = (x[sel] - cx) ** 2 + (y[sel] - cy) ** 2 + (z[sel] - cz) ** 2
        dens[sel] += per[c] * norm * np.exp(-0.5 * d2 / (sigma * sigma))
    dens = np.maximum(dens, 1.0)         # particles that strayed outside every component
    m = np.full(n, 1.0 / n)
    return Cloud("clumpy_cube", x, y, z, m, _h_from_density(dens))


def sobol_sphere(n: int = 500_000, n_neigh: int = 105, seed: int = SEED_BASE + 6) -> Cloud:
    """Quasi-random sphere (Sec. 3: a Sobol sequence filling a sphere): a
    scrambled 3-D Sobol sequence on [-1, 1]^3, points with |r| < 1 kept in
    sequence order until n are found; equal masses, h for n_neigh
    neighbours at the mean density (Table 1 uses 105)."""
    from scipy.stats import qmc
    sob = qmc.Sobol(d=3, scramble=True, seed=seed)
    pts = np.empty((0, 3))
    while pts.shape[0] < n:
        block = 2.0 * sob.random(1 << max(10, int(math.ceil(math.log2(2 * n))))) - 1.0
        pts = np.concatenate([pts, block[(block * block).sum(1) < 1.0]])
    pts = pts[:n]
    dens = np.full(n, n / (4.0 / 3.0 * math.pi))
    return Cloud("sobol_sphere", np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1]),
                 np.ascontiguousarray(pts[:, 2]), np.full(n, 1.0 / n), _h_from_density(dens, n_neigh))


def binary_clumps(n1: int = 3000, n2: int = 1000, seed: int = SEED_BASE + 7) -> Cloud:
    """A binary of two Gaussian clumps with unequal particle numbers (3000 at
    the origin, sigma 0.5; 1000 at (6, 0.3, 0), sigma 0.35), equal masses,
    h = 0.08: the case where a median split cuts the heavier clump
    (Sec. 2.1 "Load balancing")."""
    rng = np.random.default_rng(seed)
    a = 0.5 * rng.standard_normal((n1, 3))
    b = 0.35 * rng.standard_normal((n2, 3)) + np.array([6.0, 0.3, 0.0])
    p = np.concatenate([a, b])
    n = n1 + n2
    return Cloud("binary_clumps", np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]),
                 np.ascontiguousarray(p[:, 2]), np.full(n, 1.0 / n), np.full(n, 0.08))


def plummer_subset(n_sub: int = 4096, seed: int = SEED_BASE + 5,
                   parent_n: int = 1 << 20) -> Cloud:
    """Random subset of the Plummer cloud, m = 1/n_sub, h from exact kNN."""
    parent = plummer(parent_n)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(parent.n, n_sub, replace=False))
    x, y, z = parent.x[idx].copy(), parent.y[idx].copy(), parent.z[idx].copy()
    m = np.full(n_sub, 1.0 / n_sub)
    return Cloud("plummer_subset", x, y, z, m, knn_h(x, y, z))


def cotangents(n: int, seed: int = SEED_BASE + 5):
    rng = np.random.default_rng(seed + 1000)
    return rng.normal(size=n), rng.normal(size=n), rng.normal(size=n)


# Workload table: (generator, n_ll, theta values)
CONFIGS = {
    1: dict(make=uniform_sphere, n_ll=8, thetas=(0.5,), desc="N=4096 uniform unit sphere, exact-kNN h (50 neighbours), N_ll=8"),
    2: dict(make=plummer, n_ll=12, thetas=(0.5, 0.7), desc="N=2^20 Plummer (b=1, r<=20), analytic h, N_ll=12"),
    3: dict(make=plummer_background, n_ll=12, thetas=(0.7, 0.5), desc="N=2^22 Plummer + 10% uniform background (R=10.357), N_ll=12"),
    4: dict(make=clumpy_cube, n_ll=12, thetas=(0.7,), desc="unit cube, 50% uniform + 64 Gaussian clumps (sigma=0.01), N_ll=12"),
    5: dict(make=plummer, n_ll=12, thetas=(0.5, 0.7), desc="config 2 inputs + N(0,1) cotangents; 4096-particle exact-kNN subset"),
}


def small_random(n: int, seed: int, kind: str = "uniform", h_scale: float = 1.0) -> Cloud:
    """Tiny clouds for unit tests (ragged sizes, clustered shapes)."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        x, y, z = rng.uniform(-1, 1, (3, n))
    elif kind == "clustered":
        c = rng.uniform(-1, 1, (4, 3))
        lab = rng.integers(0, 4, n)
        x, y, z = (c[lab] + 0.05 * rng.normal(size=(n, 3))).T
    elif kind == "plummer":
        r = _plummer_radii(rng, n)
        x, y, z = _isotropic(rng, r)
    else:
        raise ValueError(kind)
    x, y, z = np.ascontiguousarray(x), np.ascontiguousarray(y), np.ascontiguousarray(z)
    m = rng.uniform(0.5, 1.5, n) / n
    h = h_scale * rng.uniform(0.05, 0.15, n)
    return Cloud(f"small_{kind}", x, y, z, m, h)
