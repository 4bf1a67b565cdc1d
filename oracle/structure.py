"""Structure analysis of a configuration (paper Sec. III: Voronoi coordination,
the bond-orientational order psi_6, the radial density profile), written
plainly for checking.

TEST INFRASTRUCTURE ONLY: the test suite and the smoke check are the only
callers.  The GPU library never imports anything here, and nothing here
imports the GPU library.

* ``voronoi_neighbours`` -- the Voronoi neighbours of each charge, i.e. its
  Delaunay neighbours, from scipy's Delaunay triangulation (a library
  primitive, as a sort or a matmul would be).
* ``coordination``       -- z_i, the number of Voronoi neighbours.
* ``voronoi_z``          -- the same with -2 for charges on the convex hull
  (scipy's ConvexHull), whose Voronoi cells are unbounded.
* ``psi6``               -- psi_6(i) = (1/z_i) sum over the neighbours j of
  exp(6 i theta_ij), theta_ij the angle of r_j - r_i.
* ``radial_counts``      -- counts of |r| in nbins equal bins of [0, 1]
  (bin floor(|r| nbins), clamped to the last), |r| = sqrt(x*x + y*y) rounded
  once per operation in FP64.
"""
from __future__ import annotations

import numpy as np


def voronoi_neighbours(x, y):
    """List of sorted int arrays: the Delaunay neighbours of each point."""
    from scipy.spatial import Delaunay
    pts = np.stack([np.asarray(x, np.float64), np.asarray(y, np.float64)], 1)
    tri = Delaunay(pts)
    nb = [set() for _ in range(pts.shape[0])]
    for s in tri.simplices:
        a, b, c = (int(v) for v in s)
        nb[a].update((b, c))
        nb[b].update((a, c))
        nb[c].update((a, b))
    return [np.array(sorted(v), dtype=np.int64) for v in nb]


def coordination(x, y):
    return np.array([v.size for v in voronoi_neighbours(x, y)], dtype=np.int32)


def hull_points(x, y):
    from scipy.spatial import ConvexHull
    pts = np.stack([np.asarray(x, np.float64), np.asarray(y, np.float64)], 1)
    m = np.zeros(pts.shape[0], dtype=bool)
    m[ConvexHull(pts).vertices] = True
    return m


def voronoi_z(x, y):
    z = coordination(x, y)
    z[hull_points(x, y)] = -2
    return z


def psi6(x, y, neighbours=None):
    """Complex psi_6 of each point (0 for a point without neighbours)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    if neighbours is None:
        neighbours = voronoi_neighbours(x, y)
    out = np.zeros(x.size, dtype=np.complex128)
    for i, nb in enumerate(neighbours):
        if nb.size:
            th = np.arctan2(y[nb] - y[i], x[nb] - x[i])
            out[i] = np.exp(6j * th).mean()
    return out


def radial_counts(x, y, nbins: int):
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    r = np.sqrt(x * x + y * y)
    k = np.minimum(np.floor(r * nbins), nbins - 1).astype(np.int64)
    return np.bincount(k, minlength=nbins).astype(np.int32)
