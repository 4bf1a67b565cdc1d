"""Pins of the structure oracle (no GPU): a patch of the perfect triangular
lattice (interior charges sixfold with |psi_6| = 1), an n-gon around a centre
charge (the centre n-fold, the ring threefold, psi_6 known in closed form),
and exact radial counts of charges placed on chosen radii."""
import numpy as np
import pytest

from oracle import structure as S


def tri_lattice(m):
    a, b = np.meshgrid(np.arange(-m, m + 1), np.arange(-m, m + 1), indexing="ij")
    x = (a + 0.5 * b).ravel().astype(float)
    y = (b * np.sqrt(3) / 2).ravel()
    keep = x * x + y * y <= (m * 0.8) ** 2
    return x[keep] / m, y[keep] / m


def test_triangular_lattice_interior():
    x, y = tri_lattice(12)
    z = S.coordination(x, y)
    p = np.abs(S.psi6(x, y))
    inner = np.hypot(x, y) < 0.6
    assert inner.sum() > 100
    assert (z[inner] == 6).all()
    assert np.allclose(p[inner], 1.0, atol=1e-12)
    assert z.sum() % 2 == 0  # each neighbour pair counted from both ends


@pytest.mark.parametrize("n", [5, 6, 7, 9])
def test_ngon_around_centre(n):
    t = 0.3 + 2 * np.pi * np.arange(n) / n
    x = np.append(np.cos(t), 0.0)
    y = np.append(np.sin(t), 0.0)
    z = S.coordination(x, y)
    assert z[-1] == n and (z[:-1] == 3).all()
    p = S.psi6(x, y)
    # centre: mean of exp(6 i (0.3 + 2 pi k / n)) = exp(1.8 i) if 6 is a multiple of n's
    # period, else 0: n | 6k for all k iff n divides 6
    want = np.exp(1.8j) if 6 % n == 0 else 0.0
    assert abs(p[-1] - want) < 1e-12


def test_radial_counts_exact():
    # charges on the x axis (|r| exact): bins [0,.25) [.25,.5) [.5,.75) [.75,1], |r| = 1 in the last
    r = np.array([0.0, 0.05, 0.1, 0.35, 0.5, 0.999, 1.0, 0.25])
    assert S.radial_counts(r, np.zeros(r.size), 4).tolist() == [3, 2, 1, 2]
    assert S.radial_counts(np.zeros(r.size), -r, 4).tolist() == [3, 2, 1, 2]


def test_hull_marking():
    t = 0.3 + 2 * np.pi * np.arange(8) / 8
    x = np.append(np.cos(t), 0.1)
    y = np.append(np.sin(t), 0.0)
    z = S.voronoi_z(x, y)
    assert (z[:-1] == -2).all() and z[-1] == 8
