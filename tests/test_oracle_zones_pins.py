"""Pins of the zone oracle (Sec. II.C steps 1-4) against what the mathematics
fixes (no GPU): closed-form local energies of a ring around a centre charge,
exact moments of integer data, exact lattice-point counts in a disk (Gauss's
circle problem on a dyadic grid, so every distance is exact), brute force on
tiny inputs, and the defining properties of the batch order."""
import math

import mpmath
import numpy as np
import pytest

import oracle as O
from oracle import zones as Z
from paper_2609_24722_amd import workloads as W


def ring_and_centre(n):
    t = 0.25 + 2.0 * np.pi * np.arange(n) / n
    return np.append(np.cos(t), 0.0), np.append(np.sin(t), 0.0)


def ring_centre_closed(n):
    """Local energies of n charges on the unit circle plus one at the origin:
    ring e_r = (S_n + 1)/2 with S_n = sum_k 1/(2 sin(pi k/n)); centre n/2."""
    mpmath.mp.dps = 40
    S = mpmath.fsum(1 / (2 * mpmath.sin(mpmath.pi * k / n)) for k in range(1, n))
    return (S + 1) / 2, mpmath.mpf(n) / 2


@pytest.mark.parametrize("n", [6, 200])
def test_defect_stats_ring_and_centre_closed_form(n):
    """mu and sigma_e of a two-valued distribution: mu = (n e_r + e_c)/(n+1),
    sigma_e = |e_r - e_c| sqrt(n)/(n+1).  For n = 6 the centre lies above
    the ring: kappa = -1 flags everything, kappa = +1 the centre only.  For
    n = 200 the ring lies above the centre: kappa = -1 flags the ring,
    kappa = +1 nothing."""
    x, y = ring_and_centre(n)
    _, e = O.energy(x, y, local=True)
    er, ec = ring_centre_closed(n)
    mu_c = (n * er + ec) / (n + 1)
    sg_c = abs(er - ec) * mpmath.sqrt(n) / (n + 1)
    for kappa in (-1.0, 1.0):
        mu, sg, thr, D = Z.defect_stats(e, kappa)
        assert abs(mu - float(mu_c)) <= 1e-14 * float(mu_c)
        assert abs(sg - float(sg_c)) <= 1e-11 * float(sg_c)
        assert abs(thr - float(mu_c + kappa * sg_c)) <= 1e-13 * float(mu_c)
        if n == 6:
            want = [n] if kappa > 0 else list(range(n + 1))
        else:
            want = list(range(n)) if kappa < 0 else []
        assert D.tolist() == want, (n, kappa, D)


@pytest.mark.parametrize("n", [1, 2, 10, 1001])
def test_defect_stats_integer_moments(n):
    """e = 0..n-1: mu = (n-1)/2 and sigma_e^2 = (n^2-1)/12 exactly; with
    kappa = 0 the defects are the values above the mean."""
    e = np.arange(n, dtype=np.float64)
    mu, sg, thr, D = Z.defect_stats(e, 0.0)
    assert mu == (n - 1) / 2
    assert abs(sg * sg - (n * n - 1) / 12) <= 1e-15 * max(1.0, (n * n - 1) / 12)
    assert thr == mu
    assert D.tolist() == [i for i in range(n) if i > (n - 1) / 2]
    # kappa = -1 moves the cut down by exactly one standard deviation
    _, _, thr2, D2 = Z.defect_stats(e, -1.0)
    assert D2.tolist() == [i for i in range(n) if i > mu - sg]


def test_defect_stats_constant_and_shift():
    """Constant e: sigma_e = 0 and nothing is strictly above the mean; adding
    a constant moves mu and the threshold but not sigma_e or the list."""
    mu, sg, thr, D = Z.defect_stats(np.full(17, 3.25), -1.0)
    assert (mu, sg, thr, D.size) == (3.25, 0.0, 3.25, 0)
    rng = np.random.default_rng(4)
    e = rng.normal(size=999)
    a = Z.defect_stats(e, 1.0)
    b = Z.defect_stats(e + 1024.0, 1.0)
    assert abs(b[0] - a[0] - 1024.0) < 1e-12 and abs(b[1] - a[1]) < 1e-12
    assert np.array_equal(a[3], b[3])


def test_zone_radius_triangle_wave():
    r_lo, r_hi, P = 0.05, 0.2, 10
    vals = [Z.zone_radius(t, P, r_lo, r_hi) for t in range(3 * P)]
    assert vals[0] == r_lo and vals[P] == r_lo and vals[2 * P] == r_lo
    assert abs(vals[P // 2] - r_hi) <= 2 ** -52 * r_hi
    for s in range(1, P):  # symmetric, periodic, rising then falling
        assert vals[s] == vals[P - s] == vals[s + P]
    assert all(vals[s] < vals[s + 1] for s in range(P // 2))
    # exact value of a quarter period: tri = 1/2
    assert Z.zone_radius(1, 4, 0.0, 1.0) == 0.5
    # odd period: the largest value is below r_hi
    assert max(Z.zone_radius(t, 7, 0.0, 1.0) for t in range(7)) == 6 / 7


GAUSS = {1: 5, 2: 13, 3: 29, 4: 49, 5: 81, 6: 113, 7: 149}


def test_zones_lattice_counts():
    """Square grid of spacing 1/16 (every coordinate and squared distance is
    exact): the zone of radius k/16 about a grid point holds N(k) points,
    N the lattice-point count of Gauss's circle problem (points exactly on
    the circle included)."""
    a = np.arange(-8, 9) / 16.0
    gx, gy = np.meshgrid(a, a, indexing="ij")
    x, y = gx.ravel(), gy.ravel()
    ks = sorted(GAUSS)
    ptr, idx = Z.zones(x, y, np.zeros(len(ks)), np.zeros(len(ks)), np.array(ks) / 16.0)
    assert np.diff(ptr).tolist() == [GAUSS[k] for k in ks]
    # off-grid centre (1/32, 0): radius 1/32 reaches exactly the two points (0,0), (1/16,0)
    ptr, idx = Z.zones(x, y, [1 / 32], [0.0], [1 / 32])
    assert sorted(zip(x[idx], y[idx])) == [(0.0, 0.0), (1 / 16, 0.0)]


def test_zones_brute_force():
    x, y = W.uniform_disk(300, 77)
    rng = np.random.default_rng(5)
    cx = rng.uniform(-1.2, 1.2, 9)
    cy = rng.uniform(-1.2, 1.2, 9)
    rz = np.append(rng.uniform(0.0, 0.6, 8), 0.0)
    ptr, idx = Z.zones(x, y, cx, cy, rz)
    want = []
    for c0, c1, r in zip(cx, cy, rz):
        zone = []
        for j in range(300):
            dx = float(x[j]) - float(c0)
            dy = float(y[j]) - float(c1)
            if dx * dx + dy * dy <= float(r) * float(r):
                zone.append(j)
        want.append(zone)
    assert [idx[ptr[p]:ptr[p + 1]].tolist() for p in range(9)] == want
    assert ptr[-1] - ptr[-2] == 0  # radius 0 off every charge: empty


def test_zone_centres_rule():
    x, y = W.uniform_disk(50, 8)
    D = np.array([3, 9, 27, 41], dtype=np.int32)
    draws = np.array([
        0.0, 0.0, 0.1, 0.2,        # u < p: first defect
        0.5, 0.9999999, 0.1, 0.2,  # last defect
        0.5, 0.5, 0.1, 0.2,        # floor(0.5*4) = 2
        0.8, 0.1, -0.3, 0.4,       # u = p: disk point
        0.95, 0.1, 0.6, -0.5,      # disk point
    ])
    cx, cy, ci = Z.zone_centres(x, y, D, draws, 0.8)
    assert ci.tolist() == [3, 41, 27, -1, -1]
    assert (cx[0], cy[0]) == (x[3], y[3])
    assert (cx[3], cy[3], cx[4], cy[4]) == (-0.3, 0.4, 0.6, -0.5)
    # empty list: every centre is the disk point
    cx, cy, ci = Z.zone_centres(x, y, D[:0], draws, 0.8)
    assert ci.tolist() == [-1] * 5 and cx.tolist() == draws[2::4].tolist()
    # p = 1 takes every centre from the list, p = 0 none
    d = W.zone_draws(200, 9)
    assert (Z.zone_centres(x, y, D, d, 1.0)[2] >= 0).all()
    assert (Z.zone_centres(x, y, D, d, 0.0)[2] == -1).all()
    # the share of defect centres is the share of draws u < p
    ci = Z.zone_centres(x, y, D, d, 0.8)[2]
    assert int((ci >= 0).sum()) == int((d[0::4] < 0.8).sum())


def _check_batches(cx, cy, rz, gap, cap, b, keep_order):
    """Defining properties, by brute force: no batch holds two conflicting
    zones or more than cap zones; ordered, conflicting zones keep their order
    and each zone sits in the first batch after its conflicts that had room;
    first fit, every earlier batch was full or held a conflicting zone."""
    T = len(cx)
    size = {}
    members = {}
    hit = lambda s, t: math.hypot(cx[s] - cx[t], cy[s] - cy[t]) < rz[s] + rz[t] + gap - 1e-12
    for t in range(T):
        clash = {b[s] for s in range(t) if hit(s, t)}
        assert b[t] not in clash
        if keep_order:
            need = max(clash) + 1 if clash else 0
            assert b[t] >= need
            for q in range(need, b[t]):
                assert size.get(q, 0) >= cap
        else:
            for q in range(b[t]):
                assert size.get(q, 0) >= cap or q in clash
        size[b[t]] = size.get(b[t], 0) + 1
        members.setdefault(b[t], []).append(t)
    assert max(size.values()) <= cap
    for zs in members.values():
        for i in range(len(zs)):
            for j in range(i):
                assert not hit(zs[j], zs[i])


def test_zone_batches_hand_cases():
    # a chain of overlapping zones along x, one zone far away
    cx = [0.0, 0.15, 0.3, 0.45, -0.8]
    cy = [0.0, 0.0, 0.0, 0.0, 0.0]
    rz = [0.1] * 5
    assert Z.zone_batches(cx, cy, rz, 0.0, 10).tolist() == [0, 1, 2, 3, 0]
    assert Z.zone_batches(cx, cy, rz, 0.0, 10, keep_order=False).tolist() == [0, 1, 0, 1, 0]
    # zones 0.3 apart with radii 0.1: disjoint without a gap, in conflict with gap 0.15
    cx = [0.0, 0.3, 0.6]
    assert Z.zone_batches(cx, [0.0] * 3, [0.1] * 3, 0.0, 10).tolist() == [0, 0, 0]
    assert Z.zone_batches(cx, [0.0] * 3, [0.1] * 3, 0.15, 10).tolist() == [0, 1, 2]
    assert Z.zone_batches(cx, [0.0] * 3, [0.1] * 3, 0.15, 10, keep_order=False).tolist() == [0, 1, 0]
    # capacity 1: one zone per batch, in order
    assert Z.zone_batches(cx, [0.0] * 3, [0.1] * 3, 0.0, 1).tolist() == [0, 1, 2]
    # capacity 2 with disjoint zones
    assert Z.zone_batches(cx, [0.0] * 3, [0.1] * 3, 0.0, 2).tolist() == [0, 0, 1]


@pytest.mark.parametrize("keep_order", [True, False])
@pytest.mark.parametrize("cap", [4, 1000])
def test_zone_batches_random_properties(cap, keep_order):
    rng = np.random.default_rng(11)
    T = 120
    cx = rng.uniform(-1, 1, T)
    cy = rng.uniform(-1, 1, T)
    rz = rng.uniform(0.02, 0.2, T)
    b = Z.zone_batches(cx, cy, rz, 0.01, cap, keep_order).tolist()
    _check_batches(cx.tolist(), cy.tolist(), rz.tolist(), 0.01, cap, b, keep_order)
