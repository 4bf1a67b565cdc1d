"""Seeded synthetic inputs for the unit-disk Coulomb problem.

This module only draws and lays out inputs; it computes nothing the method
computes (no energies, forces, projections or relaxations), so the CPU oracle
and the GPU path can both be fed from it.

The paper's own configurations are not available, so inputs take its sizes
and the structures the method meets (Sec. II.A: N charges in the unit disk;
Sec. II.E: subdomains of a few hundred to a few thousand active charges):

* ``uniform_disk``   -- i.i.d. uniform points in the open unit disk, drawn by
  rejection from pairs (u1, u2) ~ U[-1, 1)^2.
* ``warped_lattice`` -- a triangular lattice of spacing h with a point at the
  origin, the N points nearest the origin kept (generation order breaks ties),
  scaled into radius 1 - h/2, radially warped s -> s*sqrt(2 - s^2) so the
  uniform areal density becomes the arcsine density 1/sqrt(1 - r^2) of a
  conducting disk (introduction, below Eq. 1), then Gaussian jitter of standard
  deviation sigma*h per coordinate; a point the jitter moves outside the disk
  draws its jitter again.
* ``patch_draws``    -- subdomain centres (distinct charge indices, uniform)
  and sizes (uniform integers); the k-nearest selection itself is part of the
  method and is not done here.
* ``kicks``          -- Gaussian displacements of the active charges.
* ``zone_draws``     -- the random numbers of a cycle's zone choices: per zone
  (u, v, px, py), u and v uniform in [0, 1), (px, py) uniform in the open
  unit disk by the same rejection rule as ``uniform_disk``.

Seeds follow one rule: workload k uses 1000 + k, its secondary draws 1100 + k.
"""
from __future__ import annotations

import numpy as np


def spacing(n: int) -> float:
    """Mean triangular-lattice spacing h for n charges filling area pi."""
    return float(np.sqrt(2.0 * np.pi / (np.sqrt(3.0) * n)))


def uniform_disk(n: int, seed: int):
    rng = np.random.default_rng(seed)
    out = np.empty((0, 2))
    while out.shape[0] < n:
        u = rng.uniform(-1.0, 1.0, size=(max(2 * (n - out.shape[0]), 64), 2))
        u = u[(u * u).sum(axis=1) < 1.0]
        out = np.concatenate([out, u])
    out = out[:n]
    return np.ascontiguousarray(out[:, 0]), np.ascontiguousarray(out[:, 1])


def warped_lattice(n: int, sigma: float, seed: int):
    """Warped triangular lattice with jitter sigma*h (h = spacing(n))."""
    h = spacing(n)
    m = int(np.ceil(np.sqrt(n) * 1.2)) + 4
    a, b = np.meshgrid(np.arange(-m, m + 1), np.arange(-m, m + 1), indexing="ij")
    a = a.ravel().astype(np.float64)
    b = b.ravel().astype(np.float64)
    px = h * (a + 0.5 * b)
    py = h * (b * (np.sqrt(3.0) / 2.0))
    r2 = px * px + py * py
    order = np.argsort(r2, kind="stable")[:n]
    px = px[order]
    py = py[order]
    s = np.sqrt(px * px + py * py)
    scale = (1.0 - 0.5 * h) / s.max()
    px *= scale
    py *= scale
    s = np.sqrt(px * px + py * py)
    w = np.where(s > 0.0, np.sqrt(2.0 - s * s), 1.0)
    px *= w
    py *= w
    rng = np.random.default_rng(seed)
    x = px.copy()
    y = py.copy()
    todo = np.arange(n)
    while todo.size:
        jx = rng.normal(0.0, sigma * h, size=todo.size)
        jy = rng.normal(0.0, sigma * h, size=todo.size)
        nx = px[todo] + jx
        ny = py[todo] + jy
        ok = nx * nx + ny * ny <= 1.0
        x[todo[ok]] = nx[ok]
        y[todo[ok]] = ny[ok]
        todo = todo[~ok]
    return x, y


def unit_vector(n: int, seed: int):
    """Gaussian 2n-vector normalised to unit 2-norm, split into (vx, vy)."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 2))
    v /= np.sqrt((v * v).sum())
    return np.ascontiguousarray(v[:, 0]), np.ascontiguousarray(v[:, 1])


def patch_draws(n: int, n_patches: int, size_lo: int, size_hi: int, seed: int):
    """Distinct centre indices and sizes ~ U{size_lo..size_hi} (inclusive)."""
    rng = np.random.default_rng(seed)
    centres = rng.choice(n, size=n_patches, replace=False).astype(np.int32)
    sizes = rng.integers(size_lo, size_hi + 1, size=n_patches).astype(np.int32)
    sizes = np.minimum(sizes, n).astype(np.int32)
    return centres, sizes


def kicks(total_active: int, sigma_abs: float, seed: int):
    rng = np.random.default_rng(seed)
    k = rng.normal(0.0, sigma_abs, size=(total_active, 2))
    return np.ascontiguousarray(k[:, 0]), np.ascontiguousarray(k[:, 1])


def zone_draws(n_zones: int, seed: int) -> np.ndarray:
    """Flat float64 array [4 * n_zones] of (u, v, px, py) per zone."""
    rng = np.random.default_rng(seed)
    uv = rng.uniform(0.0, 1.0, size=(n_zones, 2))
    px, py = uniform_disk(n_zones, seed + 1) if n_zones > 0 else (np.zeros(0), np.zeros(0))
    out = np.empty((n_zones, 4))
    out[:, 0:2] = uv
    out[:, 2] = px
    out[:, 3] = py
    return np.ascontiguousarray(out.ravel())


# The five workloads, by number.  Sizes are the paper's (Sec. II.A, II.E).
def workload(k: int, n: int | None = None):
    """Positions (x, y) of workload k: 1 uniform N=1000; 2 lattice N=1e4,
    sigma 0.1h; 3 lattice N=1e5, sigma 0.02h; 4 as 3; 5 lattice sigma 0.02h at
    N=4e4 (or the given n)."""
    if k == 1:
        return uniform_disk(n or 1000, 1001)
    if k == 2:
        return warped_lattice(n or 10000, 0.1, 1002)
    if k in (3, 4):
        return warped_lattice(n or 100000, 0.02, 1003)
    if k == 5:
        return warped_lattice(n or 40000, 0.02, 1005)
    raise ValueError(f"unknown workload {k}")


def kicked_starts(x, y, idx, kx, ky):
    """Start positions of kicked candidates: snapshot positions of the packed
    charge indices plus the kicks (the relaxation projects them into the disk)."""
    idx = np.asarray(idx)
    return np.ascontiguousarray(x[idx] + kx), np.ascontiguousarray(y[idx] + ky)
