"""Pins of the oracle's (t, u) parameterisation (Sec. II.D, Eqs. 8-10) and of
its relaxation in those coordinates.

* Eqs. 8-10 against central differences of E_sub(t, u) itself (energy
  changes summed over the changed pairs, no cancellation against E).
* A closed form: n interior charges on a regular ring of radius r around the
  centre, E = E_n / r with E_n the unit ring's energy, so dE/du = 0 and
  dE/dt = -(E_n / (n r^2)) sigma sin 2t for every charge.
* The (t, u) relax reaches the same minimum as the Cartesian relax from a
  common near-minimum start (the endpoint is a property of E_sub, not of the
  coordinates), with its KKT conditions checked from the definition.
* A charge starting at the centre, where both derivatives of Eqs. 8-9 vanish,
  still moves (it keeps Cartesian coordinates).
"""
import math

import mpmath
import numpy as np

import oracle as O
from oracle import border as OB
from paper_2609_24722_amd import workloads as W


def _coords(xa, ya, kind, sigma):
    c = np.zeros(2 * xa.size)
    for a in range(xa.size):
        r = math.hypot(xa[a], ya[a])
        if kind[a] == 2:
            c[2 * a] = math.asin(math.sqrt(min(1.0, r / sigma)))
            c[2 * a + 1] = math.atan2(ya[a], xa[a])
        elif kind[a] == 1:
            c[2 * a] = math.atan2(ya[a], xa[a])
        else:
            c[2 * a], c[2 * a + 1] = xa[a], ya[a]
    return c


def _pos(c, kind, sigma):
    n = kind.size
    xa, ya = np.empty(n), np.empty(n)
    for a in range(n):
        if kind[a] == 2:
            r = sigma * math.sin(c[2 * a]) ** 2
            xa[a], ya[a] = r * math.cos(c[2 * a + 1]), r * math.sin(c[2 * a + 1])
        elif kind[a] == 1:
            xa[a], ya[a] = math.cos(c[2 * a]), math.sin(c[2 * a])
        else:
            xa[a], ya[a] = c[2 * a], c[2 * a + 1]
    return xa, ya


def test_tu_gradient_matches_central_differences():
    n = 400
    x, y = W.warped_lattice(n, 0.1, 31)
    nb = OB.boundary_count(n)
    flags = OB.border_split(x, y, nb)
    sigma = 0.97
    x, y = OB.border_spread(x, y, flags)  # the cycle's start: no near-coincident boundary charges
    x, y = OB.border_project(x, y, flags, sigma)
    r2 = x * x + y * y
    idx = np.sort(np.argsort(-r2, kind="stable")[:40]).astype(np.int32)  # charges near the edge
    idx = np.unique(np.concatenate([idx, np.argsort(r2)[:6].astype(np.int32)]))  # and near the centre
    pin = flags[idx]
    kind = np.where(pin == 1, 1, 2).astype(np.int32)
    xa, ya = x[idx], y[idx]
    c = _coords(xa, ya, kind, sigma)
    xa, ya = _pos(c, kind, sigma)
    _, gx, gy = O.esub(x, y, idx, xa, ya, grad=True)
    gc = O.tu_grad(kind, sigma, c, gx, gy)
    X = x.copy()
    Y = y.copy()
    X[idx], Y[idx] = xa, ya
    step = 1e-7
    worst = 0.0
    for a in range(idx.size):
        for k in ((0,) if kind[a] == 1 else (0, 1)):
            cp, cm = c.copy(), c.copy()
            cp[2 * a + k] += step
            cm[2 * a + k] -= step
            fd = (O.esub_delta(X, Y, idx, *_pos(cp, kind, sigma))
                  - O.esub_delta(X, Y, idx, *_pos(cm, kind, sigma))) / (2 * step)
            g = gc[2 * a + k]
            err = abs(fd - g) / max(1.0, abs(g))
            worst = max(worst, err)
            assert err <= 1e-6, (a, k, kind[a], fd, g)
    assert worst > 0.0
    assert np.all(gc[1::2][kind == 1] == 0.0)


def test_tu_gradient_closed_form_ring():
    # n charges on a ring of radius r0 < sigma, no frozen charges: E = E_n / r0
    for n in (5, 12):
        e_unit = float(mpmath.fsum((n / 2) / (2 * mpmath.sin(mpmath.pi * k / n)) for k in range(1, n)))
        sigma, r0 = 0.9, 0.6
        th = 0.37 + 2 * np.pi * np.arange(n) / n
        x, y = r0 * np.cos(th), r0 * np.sin(th)
        idx = np.arange(n, dtype=np.int32)
        kind = np.full(n, 2, dtype=np.int32)
        c = _coords(x, y, kind, sigma)
        E, gx, gy = O.esub(x, y, idx, grad=True)
        assert abs(E - e_unit / r0) <= 1e-14 * E
        gc = O.tu_grad(kind, sigma, c, gx, gy)
        t = c[0::2]
        dEdt = -(e_unit / (n * r0 * r0)) * sigma * np.sin(2 * t)
        assert np.allclose(gc[0::2], dEdt, rtol=1e-13, atol=0)
        assert np.max(np.abs(gc[1::2])) <= 1e-13 * abs(dEdt).max()


def test_tu_relax_same_minimum_as_cartesian():
    n = 3000
    x, y = W.warped_lattice(n, 0.05, 41)
    h = W.spacing(n)
    nb = OB.boundary_count(n)
    flags = OB.border_split(x, y, nb)
    sigma = 1.0 - 1.0 / (2.0 * math.sqrt(n))
    x, y = OB.border_spread(x, y, flags)
    x, y = OB.border_project(x, y, flags, sigma)
    for centre in (int(np.argmax(x * x + y * y)), int(np.argmin(x * x + y * y))):
        idx = O.patches(x, y, [centre], [60])
        pin = flags[idx]
        xa0, ya0, st0 = O.relax(x, y, idx, pin=pin, sigma=sigma, gtol=1e-8, max_iter=20000)
        assert st0["status"] == 0
        rng = np.random.default_rng(centre)
        sx = xa0 + rng.normal(0, 1e-3 * h, idx.size)
        sy = ya0 + rng.normal(0, 1e-3 * h, idx.size)
        xa, ya, st = O.relax_tu(x, y, idx, sx, sy, pin=pin, sigma=sigma, gtol=1e-8)
        xb, yb, stb = O.relax(x, y, idx, sx, sy, pin=pin, sigma=sigma, gtol=1e-8, max_iter=20000)
        assert st["status"] == 0 and stb["status"] == 0
        Ea = O.esub(x, y, idx, xa, ya)
        Eb = O.esub(x, y, idx, xb, yb)
        assert abs(Ea - Eb) <= 1e-12 * abs(Eb)
        assert np.hypot(xa - xb, ya - yb).max() <= 1e-3 * h
        # KKT from the definition: boundary charges on the circle, interior
        # within sigma, reduced gradient below the tolerance
        r = np.hypot(xa, ya)
        assert np.all(np.abs(r[pin == 1] - 1.0) <= 1e-15)
        assert np.all(r[pin == 0] <= sigma * (1 + 1e-15))
        _, gx, gy = O.esub(x, y, idx, xa, ya, grad=True)
        assert O.reduce_grad(xa, ya, gx, gy, pin=pin, sigma=sigma)[3] <= 1e-8


def test_tu_relax_moves_a_charge_from_the_centre():
    # at r = 0 both derivatives of Eqs. 8-9 vanish for any force: the charge
    # keeps Cartesian coordinates.  Six frozen charges on a ring of radius
    # 0.3 about (0.02, 0.01) make that point its minimum (by symmetry); the
    # charge starts at the disk's centre and must reach it
    c0 = np.array([0.02, 0.01])
    th = 2 * np.pi * np.arange(6) / 6 + 0.1
    x = np.concatenate([[0.0], c0[0] + 0.3 * np.cos(th)])
    y = np.concatenate([[0.0], c0[1] + 0.3 * np.sin(th)])
    idx = np.array([0], dtype=np.int32)
    xa, ya, st = O.relax_tu(x, y, idx, sigma=1.0, gtol=1e-10, step0=0.005)
    assert st["status"] == 0
    assert math.hypot(xa[0] - c0[0], ya[0] - c0[1]) <= 1e-10
