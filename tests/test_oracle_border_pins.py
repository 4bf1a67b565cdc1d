"""Pins of the border-interior oracle (Sec. II.B) against what the paper and
the mathematics fix (no GPU): Table I's optimal boundary population at
N = 1e5, minima known in closed form under the pinned-boundary and
interior-wall constraint, the KKT conditions of its endpoints, brute force
for the boundary split, and the identity with the hard wall at sigma = 1."""
import math

import mpmath
import numpy as np
import pytest

import oracle as O
from oracle import border as B
from paper_2609_24722_amd import workloads as W


def ngon_energy(n, radius=1.0):
    mpmath.mp.dps = 40
    e = mpmath.mpf(n) / 2 * mpmath.fsum(1 / (2 * mpmath.sin(mpmath.pi * k / n)) for k in range(1, n))
    return float(e / radius)


def test_boundary_count_table_one():
    """Table I: at N = 1e5 the lowest energy has N_b = 6099 (N_core = 93901),
    which the text says agrees with Eq. 4."""
    assert B.boundary_count(100000) == 6099
    assert 100000 - B.boundary_count(100000) == 93901
    # increasing in N, and about 2.8 N^(2/3) for large N
    v = [B.boundary_count(n) for n in (100, 1000, 10000, 40000, 100000)]
    assert v == sorted(v) and all(a < b for a, b in zip(v, v[1:]))


def test_sigma_schedule():
    assert B.sigma0(100) == 0.95
    assert B.sigma0(10000) == 0.995
    assert B.sigma_ramp(0, 4, 10000) == B.sigma0(10000) and B.sigma_ramp(4, 4, 10000) == 1.0
    vals = [B.sigma_ramp(k, 4, 10000) for k in range(5)]
    assert all(a < b for a, b in zip(vals, vals[1:]))


def test_border_split_brute_force():
    x, y = W.uniform_disk(200, 31)
    # an exact tie in x*x + y*y: two charges on the same circle
    x[10], y[10] = 0.6, 0.8
    x[20], y[20] = 0.8, 0.6
    r2 = [float(a) * float(a) + float(b) * float(b) for a, b in zip(x, y)]
    for nb in (0, 1, 37, 200):
        f = B.border_split(x, y, nb)
        assert f.sum() == nb
        want = sorted(range(200), key=lambda i: (-r2[i], i))[:nb]
        assert sorted(np.nonzero(f)[0].tolist()) == sorted(want)


def _relax_all(x, y, pin, sigma, gtol=1e-11):
    idx = np.arange(x.size, dtype=np.int32)
    xa, ya, st = O.relax(x, y, idx, x.copy(), y.copy(), gtol=gtol, pin=pin, sigma=sigma)
    return xa, ya, st


def test_relax_bi_hexagon_and_centre():
    """Six pinned charges and one interior charge (sigma = 0.5): the minimum is
    the regular hexagon on the unit circle with the seventh charge at the
    centre, E = E_6 + 6."""
    t = np.arange(6) * (2 * np.pi / 6) + np.array([0.1, -0.05, 0.08, 0.0, -0.1, 0.03])
    x = np.append(np.cos(t) * 0.9, 0.2)   # the projection puts pinned charges on the circle
    y = np.append(np.sin(t) * 0.9, -0.1)
    pin = np.array([1] * 6 + [0], dtype=np.int32)
    xa, ya, st = _relax_all(x, y, pin, 0.5)
    assert st["status"] == 0
    assert abs(O.energy(xa, ya) - (ngon_energy(6) + 6.0)) < 1e-12
    assert np.allclose(np.hypot(xa[:6], ya[:6]), 1.0, atol=1e-15)
    assert np.hypot(xa[6], ya[6]) < 1e-9


def test_relax_bi_interior_wall_triangle():
    """Three interior charges with the wall at sigma: they sit on the sigma
    circle as an equilateral triangle, E = sqrt(3) / sigma, all held."""
    x = np.array([0.1, -0.2, 0.05])
    y = np.array([0.1, 0.0, -0.3])
    for sigma in (0.5, 0.9):
        xa, ya, st = _relax_all(x, y, np.zeros(3, dtype=np.int32), sigma)
        assert st["status"] == 0
        assert abs(O.energy(xa, ya) - math.sqrt(3.0) / sigma) < 1e-12
        assert np.allclose(np.hypot(xa, ya), sigma, atol=1e-14)
        # the forces point outward at the wall; reduce_grad takes the gradient (-F)
        _, _, held, gi = O.reduce_grad(xa, ya, *[-f for f in O.forces(xa, ya)], pin=np.zeros(3, np.int32),
                                       sigma=sigma)
        assert held.tolist() == [1, 1, 1] and gi < 1e-10


@pytest.mark.parametrize("n", [5, 9])
def test_relax_bi_all_pinned_ngon(n):
    """Every charge pinned: the minimum on the circle is the regular n-gon."""
    t = np.sort(np.random.default_rng(n).uniform(0, 2 * np.pi, n))
    x, y = 0.7 * np.cos(t), 0.7 * np.sin(t)
    xa, ya, st = _relax_all(x, y, np.ones(n, dtype=np.int32), 0.3)
    assert st["status"] == 0
    assert abs(O.energy(xa, ya) - ngon_energy(n)) < 1e-12 * ngon_energy(n)
    assert np.allclose(np.hypot(xa, ya), 1.0, atol=1e-15)


def test_relax_bi_reduces_to_hard_wall():
    """No pinned charge and sigma = 1: the same path as the hard wall of Eq. 3."""
    x, y = W.uniform_disk(40, 7)
    idx = np.arange(40, dtype=np.int32)
    a = O.relax(x, y, idx, x.copy(), y.copy(), gtol=1e-9)
    b = O.relax(x, y, idx, x.copy(), y.copy(), gtol=1e-9, pin=np.zeros(40, np.int32), sigma=1.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_relax_bi_kkt_endpoint():
    """A border-interior relax of a 60-charge disk: boundary charges on the
    circle, interior ones inside sigma, held interior charges pushed outward,
    reduced gradient below the tolerance (checked with the hard-wall-free
    reduction computed here from the definition)."""
    n = 60
    x, y = W.uniform_disk(n, 12)
    nb = 20
    pin = B.border_split(x, y, nb)
    sigma = 0.9
    xa, ya, st = _relax_all(x, y, pin, sigma, gtol=1e-9)
    assert st["status"] == 0
    fx, fy = O.forces(xa, ya)
    gx, gy = -fx, -fy
    r = np.hypot(xa, ya)
    assert np.allclose(r[pin == 1], 1.0, atol=1e-15)
    assert (r[pin == 0] <= sigma * (1 + 1e-15)).all()
    worst = 0.0
    for a in range(n):
        ux, uy = xa[a] / r[a], ya[a] / r[a]
        gr = gx[a] * ux + gy[a] * uy
        if pin[a] or (r[a] >= sigma * (1 - 1e-14) and gr < 0):
            tx, ty = gx[a] - gr * ux, gy[a] - gr * uy
        else:
            tx, ty = gx[a], gy[a]
        worst = max(worst, abs(tx), abs(ty))
    assert worst <= 1e-9
    assert ((r >= sigma * (1 - 1e-14)) & (pin == 0)).sum() > 0  # the interior wall is active


def test_border_project_definition():
    """Projection: boundary charges land on the unit circle along their ray,
    interior charges beyond sigma on the sigma circle, the rest unchanged
    (dyadic points make every value exact)."""
    x = np.array([0.5, 0.0, 0.75, 0.25, -0.5])
    y = np.array([0.0, 0.5, 0.0, 0.0, 0.0])
    flags = np.array([1, 1, 0, 0, 0])
    px, py = B.border_project(x, y, flags, 0.5)
    assert px.tolist() == [1.0, 0.0, 0.5, 0.25, -0.5] and py.tolist() == [0.0, 1.0, 0.0, 0.0, 0.0]
    x, y = W.uniform_disk(500, 3)
    px, py = B.border_project(x, y, None, 0.7)
    r0, r1 = np.hypot(x, y), np.hypot(px, py)
    assert np.all(r1 <= 0.7 * (1 + 1e-15)) and np.array_equal(px[r0 <= 0.7], x[r0 <= 0.7])
    assert np.allclose(np.arctan2(py, px), np.arctan2(y, x), atol=1e-15)


def test_border_spread_pins():
    # a regular nb-gon on the circle, listed in shuffled order among interior
    # charges: spreading returns it unchanged (to rounding); the angular
    # order of any boundary set is kept and the spacing is exactly 2 pi / nb
    rng = np.random.default_rng(5)
    nb = 37
    phi = 0.3 + 2 * np.pi * np.arange(nb) / nb
    bx, by = np.cos(phi), np.sin(phi)
    ix = rng.uniform(-0.5, 0.5, 20)
    iy = rng.uniform(-0.5, 0.5, 20)
    perm = rng.permutation(nb + 20)
    x = np.concatenate([bx, ix])[perm]
    y = np.concatenate([by, iy])[perm]
    flags = (perm < nb).astype(np.int32)
    sx, sy = B.border_spread(x, y, flags)
    assert np.allclose(sx, x, atol=1e-15, rtol=0) and np.allclose(sy, y, atol=1e-15, rtol=0)
    assert np.array_equal(sx[flags == 0], x[flags == 0]) and np.array_equal(sy[flags == 0], y[flags == 0])
    # charges of three rings on common rays (the unrelaxed lattice's outer
    # rings): after spreading every neighbour distance is the chord 2 sin(pi/nb)
    rays = np.repeat(np.arange(12) * 2 * np.pi / 12, 3)
    rad = np.tile([0.97, 0.985, 1.0], 12)
    x, y = rad * np.cos(rays), rad * np.sin(rays)
    fl = np.ones(36, dtype=np.int32)
    sx, sy = B.border_spread(x, y, fl)
    assert np.allclose(np.hypot(sx, sy), 1.0, atol=1e-15, rtol=0)
    th = np.sort(np.mod(np.arctan2(sy, sx), 2 * np.pi))
    gaps = np.diff(np.concatenate([th, [th[0] + 2 * np.pi]]))
    assert np.allclose(gaps, 2 * np.pi / 36, atol=1e-13, rtol=0)
    # the order: ties in angle (a ray) go to the lower index first
    k = np.argsort(np.lexsort((np.arange(36), np.arctan2(y, x))))
    ang = np.mod(np.arctan2(sy, sx) - np.arctan2(sy[np.argmin(k)], sx[np.argmin(k)]), 2 * np.pi)
    assert np.array_equal(np.argsort(ang, kind="stable"), np.argsort(k, kind="stable"))
    # nothing flagged: unchanged
    sx, sy = B.border_spread(x, y, np.zeros(36, dtype=np.int32))
    assert np.array_equal(sx, x) and np.array_equal(sy, y)
