"""Pins of the Riesz-s oracle (no GPU): regular n-gons in closed form for
s = 2 and s = 4 (sums of csc^2 and csc^4), an mpmath sum for other s, the
Coulomb case s = 1 through the separately pinned 1/r routines, Euler's
identity for a homogeneous energy (sum r.F = s E), and forces against
energy differences."""
import mpmath
import numpy as np
import pytest

import oracle as O
from paper_2609_24722_amd import workloads as W


def ngon(n, phase=0.2):
    t = phase + 2 * np.pi * np.arange(n) / n
    return np.cos(t), np.sin(t)


@pytest.mark.parametrize("n", [2, 3, 7, 16, 101])
def test_ngon_closed_forms(n):
    x, y = ngon(n)
    # sum_k csc^2(pi k/n) = (n^2-1)/3, sum_k csc^4(pi k/n) = (n^2-1)(n^2+11)/45; chords 2 sin(pi k/n)
    assert abs(O.riesz(x, y, 2.0, False) - n * (n * n - 1) / 24) <= 1e-13 * n ** 3
    assert abs(O.riesz(x, y, 4.0, False) - n * (n * n - 1) * (n * n + 11) / 1440) <= 1e-13 * n ** 5


@pytest.mark.parametrize("s", [0.5, 1.7, 3.0])
def test_ngon_general_s(s):
    n = 23
    x, y = ngon(n)
    mpmath.mp.dps = 40
    want = mpmath.mpf(n) / 2 * mpmath.fsum((2 * mpmath.sin(mpmath.pi * k / n)) ** (-s) for k in range(1, n))
    assert abs(O.riesz(x, y, s, False) - float(want)) <= 1e-13 * float(want)


def test_coulomb_case():
    x, y = W.uniform_disk(300, 5)
    E, fx, fy = O.riesz(x, y, 1.0)
    assert abs(E - O.energy(x, y)) <= 1e-13 * E
    gx, gy = O.forces(x, y)
    assert np.sqrt(np.sum((fx - gx) ** 2 + (fy - gy) ** 2) / np.sum(gx ** 2 + gy ** 2)) < 1e-13


@pytest.mark.parametrize("s", [0.5, 2.0, 3.5])
def test_euler_and_finite_differences(s):
    # a jittered lattice: no near-coincident pair, so E stays small enough for
    # central differences
    x, y = W.warped_lattice(120, 0.1, 6)
    E, fx, fy = O.riesz(x, y, s)
    assert abs(np.sum(x * fx + y * fy) - s * E) <= 1e-11 * s * E
    h = 1e-6
    for i in (0, 57):
        for comp in (0, 1):
            xp, yp, xm, ym = x.copy(), y.copy(), x.copy(), y.copy()
            if comp == 0:
                xp[i] += h
                xm[i] -= h
            else:
                yp[i] += h
                ym[i] -= h
            fd = -(O.riesz(xp, yp, s, False) - O.riesz(xm, ym, s, False)) / (2 * h)
            f = fx[i] if comp == 0 else fy[i]
            assert abs(fd - f) <= 1e-5 * max(1.0, abs(f))
