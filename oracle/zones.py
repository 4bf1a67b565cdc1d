"""Defect-targeted zones of the subdomain cycle, written plainly for checking.

TEST INFRASTRUCTURE ONLY: the test suite and the smoke check are the only
callers.  The GPU library never imports anything here, and nothing here
imports the GPU library.

What it computes (paper Sec. II.C, steps 1-4 and the closing paragraph on the
zone radius):

* ``defect_stats`` -- from the local energies e_i (step 1, ``energy(...,
  local=True)`` in this package), the mean mu and the standard deviation
  sigma_e of their distribution, the threshold mu + kappa*sigma_e and the
  list of charges above it (step 2).
* ``zone_radius``  -- the zone radius of the t-th zone of a cycle: it
  oscillates periodically between r_lo and r_hi.
* ``zone_centres`` -- the centre of each zone (step 3): with probability
  p_defect a defect charge chosen uniformly from the list, otherwise a point
  drawn uniformly over the disk.
* ``zones``        -- the active set of each zone: every charge within the
  zone radius of its centre (step 4).
* ``zone_batches`` -- batches of zones a GPU may relax side by side: no two
  zones of a batch come within ``gap`` of each other, batches hold at most
  ``cap`` zones; in sequence order either after every earlier conflicting
  zone (order kept) or in the first batch free of conflicts (first fit).

Readings where the paper is silent or ambiguous:

* sigma_e is the population standard deviation (divide by n).  Sums are
  exact (math.fsum), then each operation is rounded once in FP64.
* Step 2 prints the threshold as mu minus sigma_e; kappa = -1 is that literal
  reading, kappa = +1 the alternative that flags a high-energy tail.  A charge
  is a defect iff e_i > threshold (strict).
* A defect centre is list[min(floor(v * |list|), |list| - 1)] for a uniform
  v in [0, 1); with an empty list every centre is a disk point.
* The radius oscillation is a triangle wave over the zone index t:
  s = t mod period, tri = 2 min(s, period - s) / period (0 at s = 0, 1 at
  s = period / 2), r = r_lo + (r_hi - r_lo) * tri.
* Membership is |r_j - c|^2 <= r^2 with (dx*dx) + (dy*dy) and r*r each
  rounded in FP64 (no fused multiply-add).
* Two zones conflict iff (cx_a - cx_b)^2 + (cy_a - cy_b)^2 <
  (r_a + r_b + gap)^2, rounded the same way.

Every random number is an input (``draws``): per zone four doubles
(u, v, px, py), u and v uniform in [0, 1) and (px, py) uniform in the disk.
"""
from __future__ import annotations

import math

import numpy as np


def defect_stats(e, kappa: float):
    """Returns (mu, sigma_e, threshold, defect list int32 in increasing index
    order) for local energies e (Sec. II.C step 2)."""
    e = np.asarray(e, dtype=np.float64)
    n = e.size
    mu = math.fsum(e.tolist()) / n
    dev = e - mu
    var = math.fsum((dev * dev).tolist()) / n
    sigma = math.sqrt(var)
    thr = mu + kappa * sigma
    D = np.nonzero(e > thr)[0].astype(np.int32)
    return mu, sigma, thr, D


def zone_radius(t: int, period: int, r_lo: float, r_hi: float) -> float:
    """Radius of zone t: triangle wave of the given period between r_lo and r_hi."""
    s = t % period
    m = min(s, period - s)
    tri = float(2 * m) / float(period)
    return r_lo + (r_hi - r_lo) * tri


def zone_centres(x, y, D, draws, p_defect: float):
    """Centres (cx, cy) and the charge index of each centre (-1 for a disk
    point) of len(draws) // 4 zones (Sec. II.C step 3)."""
    draws = np.asarray(draws, dtype=np.float64).reshape(-1, 4)
    P = draws.shape[0]
    cx = np.empty(P)
    cy = np.empty(P)
    ci = np.empty(P, dtype=np.int32)
    nd = len(D)
    for t in range(P):
        u, v, px, py = (float(a) for a in draws[t])
        if u < p_defect and nd > 0:
            k = min(int(math.floor(v * nd)), nd - 1)
            i = int(D[k])
            cx[t], cy[t], ci[t] = x[i], y[i], i
        else:
            cx[t], cy[t], ci[t] = px, py, -1
    return cx, cy, ci


def zones(x, y, cx, cy, rz):
    """Active sets: zone p holds every charge j with |r_j - c_p| <= rz[p],
    in increasing index order.  Returns (ptr int32 [P+1], idx int32)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    parts = []
    for c0, c1, r in zip(np.asarray(cx, dtype=np.float64), np.asarray(cy, dtype=np.float64),
                         np.asarray(rz, dtype=np.float64)):
        dx = x - c0
        dy = y - c1
        d2 = dx * dx + dy * dy
        parts.append(np.nonzero(d2 <= r * r)[0])
    ptr = np.zeros(len(parts) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([p.size for p in parts])
    idx = np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)
    return ptr.astype(np.int32), idx.astype(np.int32)


def conflict(ax, ay, ar, bx, by, br, gap: float) -> bool:
    dx = ax - bx
    dy = ay - by
    reach = ar + br + gap
    return dx * dx + dy * dy < reach * reach


def zone_batches(cx, cy, rz, gap: float, cap: int, keep_order: bool = True):
    """Batch index of each zone, zones taken in sequence order.  keep_order:
    the first batch after those of all earlier conflicting zones; otherwise
    the first batch holding no zone in conflict with it (first fit).  Either
    way batches already holding cap zones are passed over."""
    cx = [float(a) for a in cx]
    cy = [float(a) for a in cy]
    rz = [float(a) for a in rz]
    batch = []
    members = {}
    for t in range(len(cx)):
        clash = set()
        for s in range(t):
            if conflict(cx[s], cy[s], rz[s], cx[t], cy[t], rz[t], gap):
                clash.add(batch[s])
        b = (max(clash) + 1 if clash else 0) if keep_order else 0
        while len(members.get(b, [])) >= cap or (not keep_order and b in clash):
            b += 1
        batch.append(b)
        members.setdefault(b, []).append(t)
    return np.asarray(batch, dtype=np.int32)
