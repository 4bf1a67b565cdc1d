"""Border-interior decomposition (paper Sec. II.B), written plainly for checking.

TEST INFRASTRUCTURE ONLY: the test suite and the smoke check are the only
callers.  The GPU library never imports anything here, and nothing here
imports the GPU library.

* ``boundary_count`` -- N_b of Eq. 4, rounded to the nearest integer.
* ``sigma0``         -- the initial interior radius of Eq. 5.
* ``sigma_ramp``     -- the interior radius at stage k of K, rising linearly
  from sigma0 to 1 (the paper names the end points, not the law).
* ``border_split``   -- which charges are boundary charges: the N_b charges
  farthest from the centre, by x*x + y*y rounded once per operation in FP64,
  ties to the lower index.
* ``border_project`` -- the feasible point nearest along the ray: boundary
  charges onto the unit circle (x / r), others beyond sigma onto radius sigma
  (x * (sigma / r)).
* ``border_spread``  -- the start of the split used before a cycle (a step
  the paper leaves open): the boundary charges onto the unit circle, evenly
  spaced in angle in their angular order, so that charges of adjacent rings
  on one ray do not land on top of each other.

The relaxation under this constraint is ``relax(..., pin=..., sigma=...)`` of
this package (oracle.c: boundary charges pinned to the unit circle, the others
confined to |r| <= sigma).
"""
from __future__ import annotations

import math

import numpy as np


def boundary_count(n: int) -> int:
    """Eq. 4: N_b = 2.84328 N^(2/3) - 0.530196 N^(1/3) - 2.32866, nearest integer."""
    c = float(n) ** (1.0 / 3.0)
    return int(math.floor(2.84328 * c * c - 0.530196 * c - 2.32866 + 0.5))


def sigma0(n: int) -> float:
    """Eq. 5: sigma = 1 - 1 / (2 sqrt(N))."""
    return 1.0 - 1.0 / (2.0 * math.sqrt(n))


def sigma_ramp(k: int, stages: int, n: int) -> float:
    """Interior radius of stage k = 0..stages: sigma0 + (1 - sigma0) k / stages."""
    s0 = sigma0(n)
    return s0 + (1.0 - s0) * (k / stages) if stages > 0 else 1.0


def border_split(x, y, nb: int) -> np.ndarray:
    """int32 flags [N]: 1 for the nb charges with the largest x*x + y*y (ties
    to the lower index), 0 for the others."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r2 = x * x + y * y
    order = np.lexsort((np.arange(x.size), -r2))  # largest first, then lower index
    flags = np.zeros(x.size, dtype=np.int32)
    flags[order[:nb]] = 1
    return flags


def border_project(x, y, flags, sigma: float):
    """Projected copies of (x, y) (see the module docstring)."""
    x = np.array(x, dtype=np.float64, copy=True)
    y = np.array(y, dtype=np.float64, copy=True)
    r = np.sqrt(x * x + y * y)
    fl = np.zeros(x.size, bool) if flags is None else np.asarray(flags) != 0
    on = fl & (r > 0.0)
    x[on] = x[on] / r[on]
    y[on] = y[on] / r[on]
    out = ~fl & (r > sigma)
    f = sigma / r[out]
    x[out] = x[out] * f
    y[out] = y[out] * f
    return x, y


def border_spread(x, y, flags):
    """Copies of (x, y) with the flagged charges moved onto the unit circle:
    ordered by theta = atan2(y, x) (ties to the lower index), the k-th of the
    nb flagged charges goes to angle theta_0 + 2 pi k / nb, theta_0 the angle
    of the first.  Unflagged charges are unchanged."""
    x = np.array(x, dtype=np.float64, copy=True)
    y = np.array(y, dtype=np.float64, copy=True)
    idx = np.flatnonzero(np.asarray(flags) != 0)
    nb = idx.size
    if nb == 0:
        return x, y
    th = np.arctan2(y[idx], x[idx])
    order = idx[np.lexsort((idx, th))]  # by angle, then index
    th0 = float(np.arctan2(y[order[0]], x[order[0]]))
    for k, i in enumerate(order):
        phi = th0 + 2.0 * math.pi * k / nb
        x[i] = math.cos(phi)
        y[i] = math.sin(phi)
    return x, y
