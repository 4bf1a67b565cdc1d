"""CPU FP64 oracle for the unit-disk Coulomb problem.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library never imports or
links anything here, and nothing here imports the GPU library.

The arithmetic lives in ``oracle.c`` (plain C, FP64, Neumaier-compensated sums
in a fixed order, OpenMP over rows).  This module is argument marshalling plus
a few dense linear-algebra helpers built from numpy primitives:

* ``tangent_hessian_dense`` -- the Hessian of the energy restricted to the
  feasible tangent space of the hard wall (Eq. 3), with the curvature term of
  the circle for charges held by the wall; used to pin the GPU Lanczos
  certificate at small N via ``numpy.linalg.eigh``.

Paper passages: Eq. 2 (pair energy), Eq. 3 (hard wall), Eqs. 6-7 (subdomain
objective), Sec. II.C step 1 (local energies), step 4 (local relaxation).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)


class RelaxOpts(ctypes.Structure):
    _fields_ = [
        ("max_iter", ctypes.c_int32),
        ("lbfgs_m", ctypes.c_int32),
        ("gtol", ctypes.c_double),
        ("newton_tol", ctypes.c_double),
        ("step0", ctypes.c_double),
        ("cg_max", ctypes.c_int32),
    ]


class RelaxStats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("newton_steps", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("gtan_inf", ctypes.c_double),
    ]


def build() -> str:
    """Compile liboracle.so with gcc (IEEE FP64: no fast-math, no contraction)."""
    cmd = [
        "gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-ffp-contract=off", "-fPIC",
        "-shared", _SRC, "-o", _LIB + ".tmp", "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_energy.restype = ctypes.c_double
        L.orc_energy.argtypes = [ctypes.c_int64, _D, _D, _D]
        L.orc_riesz.restype = ctypes.c_double
        L.orc_riesz.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_double, _D, _D]
        L.orc_forces.restype = None
        L.orc_forces.argtypes = [ctypes.c_int64, _D, _D, _D, _D]
        L.orc_hvp.restype = None
        L.orc_hvp.argtypes = [ctypes.c_int64, _D, _D, _D, _D, _D, _D]
        L.orc_hessian.restype = None
        L.orc_hessian.argtypes = [ctypes.c_int64, _D, _D, _D]
        L.orc_esub.restype = ctypes.c_double
        L.orc_esub.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_int64, _I32, _D, _D, _D, _D]
        L.orc_esub_delta.restype = ctypes.c_double
        L.orc_esub_delta.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_int64, _I32, _D, _D]
        L.orc_esub_hvp.restype = None
        L.orc_esub_hvp.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_int64, _I32, _D, _D, _D, _D, _D, _D]
        L.orc_reduce_grad.restype = ctypes.c_double
        L.orc_reduce_grad.argtypes = [ctypes.c_int64, _D, _D, _D, _D, _D, _D, _I32]
        L.orc_reduce_grad_bi.restype = ctypes.c_double
        L.orc_reduce_grad_bi.argtypes = [ctypes.c_int64, _D, _D, _D, _D, _I32, ctypes.c_double, _D, _D, _I32]
        L.orc_relax_bi.restype = None
        L.orc_relax_bi.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_int64, _I32, _I32, ctypes.c_double, _D, _D,
                                   ctypes.POINTER(RelaxOpts), ctypes.POINTER(RelaxStats)]
        L.orc_relax_tu.restype = None
        L.orc_relax_tu.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_int64, _I32, _I32, ctypes.c_double, _D, _D,
                                   ctypes.POINTER(RelaxOpts), ctypes.POINTER(RelaxStats)]
        L.orc_tu_grad.restype = None
        L.orc_tu_grad.argtypes = [ctypes.c_int64, _I32, ctypes.c_double, _D, _D, _D, _D]
        L.orc_relax.restype = None
        L.orc_relax.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_int64, _I32, _D, _D,
                                ctypes.POINTER(RelaxOpts), ctypes.POINTER(RelaxStats)]
        L.orc_rows.restype = None
        L.orc_rows.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_int64, _I32, _D, _D, _D]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I32)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def energy(x, y, local: bool = False):
    """E = sum_{i<j} 1/r_ij (Eq. 2); with local=True also e_i (Sec. II.C step 1)."""
    x, px = _d(x)
    y, py = _d(y)
    n = x.size
    if local:
        e = np.empty(n)
        E = lib().orc_energy(n, px, py, e.ctypes.data_as(_D))
        return E, e
    return lib().orc_energy(n, px, py, None)


def forces(x, y):
    """F_i = -dE/dr_i = sum_{j!=i} (r_i - r_j)/r_ij^3."""
    x, px = _d(x)
    y, py = _d(y)
    fx = np.empty(x.size)
    fy = np.empty(x.size)
    lib().orc_forces(x.size, px, py, fx.ctypes.data_as(_D), fy.ctypes.data_as(_D))
    return fx, fy


def riesz(x, y, s: float, forces: bool = True):
    """Riesz-s energy sum_{i<j} r^-s and, with forces, F_i = sum_j s (r_i - r_j)
    r^(-s-2).  Returns E or (E, fx, fy)."""
    x, px = _d(x)
    y, py = _d(y)
    n = x.size
    if not forces:
        return lib().orc_riesz(n, px, py, float(s), None, None)
    fx = np.empty(n)
    fy = np.empty(n)
    E = lib().orc_riesz(n, px, py, float(s), fx.ctypes.data_as(_D), fy.ctypes.data_as(_D))
    return E, fx, fy


def hvp(x, y, vx, vy):
    """(H v)_i = sum_{j!=i} K(d_ij)(v_i - v_j), K(d) = (3dd^T - |d|^2 I)/|d|^5."""
    x, px = _d(x)
    y, py = _d(y)
    vx, pvx = _d(vx)
    vy, pvy = _d(vy)
    hx = np.empty(x.size)
    hy = np.empty(x.size)
    lib().orc_hvp(x.size, px, py, pvx, pvy, hx.ctypes.data_as(_D), hy.ctypes.data_as(_D))
    return hx, hy


def rows(x, y, rows, vx=None, vy=None):
    """F_i (or (H v)_i if v is given) and e_i for the charges in ``rows``."""
    x, px = _d(x)
    y, py = _d(y)
    rows, pr = _i(rows)
    pvx = pvy = None
    if vx is not None:
        vx, pvx = _d(vx)
        vy, pvy = _d(vy)
    o0 = np.empty(rows.size)
    o1 = np.empty(rows.size)
    e = np.empty(rows.size)
    lib().orc_rows(x.size, px, py, pvx, pvy, rows.size, pr, o0.ctypes.data_as(_D),
                   o1.ctypes.data_as(_D), e.ctypes.data_as(_D))
    return o0, o1, e


def hessian(x, y):
    """Dense 2N x 2N Hessian of E, coordinates ordered (x0, y0, x1, y1, ...)."""
    x, px = _d(x)
    y, py = _d(y)
    H = np.empty((2 * x.size, 2 * x.size))
    lib().orc_hessian(x.size, px, py, H.ctypes.data_as(_D))
    return H


def esub(x, y, idx, xa=None, ya=None, grad: bool = False):
    """Subdomain objective of Eqs. 6-7 with active set ``idx`` moved to (xa, ya)."""
    x, px = _d(x)
    y, py = _d(y)
    idx, pidx = _i(idx)
    na = idx.size
    pxa = pya = None
    if xa is not None:
        xa, pxa = _d(xa)
        ya, pya = _d(ya)
    if grad:
        gx = np.empty(na)
        gy = np.empty(na)
        E = lib().orc_esub(x.size, px, py, na, pidx, pxa, pya, gx.ctypes.data_as(_D), gy.ctypes.data_as(_D))
        return E, gx, gy
    return lib().orc_esub(x.size, px, py, na, pidx, pxa, pya, None, None)


def esub_delta(x, y, idx, xa, ya):
    """E_sub(active at (xa, ya)) - E_sub(active at the snapshot), pair by pair."""
    x, px = _d(x)
    y, py = _d(y)
    idx, pidx = _i(idx)
    xa, pxa = _d(xa)
    ya, pya = _d(ya)
    return lib().orc_esub_delta(x.size, px, py, idx.size, pidx, pxa, pya)


def esub_hvp(x, y, idx, xa, ya, vx, vy):
    x, px = _d(x)
    y, py = _d(y)
    idx, pidx = _i(idx)
    pxa = pya = None
    if xa is not None:
        xa, pxa = _d(xa)
        ya, pya = _d(ya)
    vx, pvx = _d(vx)
    vy, pvy = _d(vy)
    hx = np.empty(idx.size)
    hy = np.empty(idx.size)
    lib().orc_esub_hvp(x.size, px, py, idx.size, pidx, pxa, pya, pvx, pvy,
                       hx.ctypes.data_as(_D), hy.ctypes.data_as(_D))
    return hx, hy


def reduce_grad(xa, ya, gx, gy, pin=None, sigma: float = 1.0):
    """KKT reduction of the gradient: returns (tx, ty, held, inf_norm).
    Hard wall of Eq. 3 by default; with pin (flags per charge) and sigma the
    border-interior constraint of Sec. II.B (pinned charges on the unit
    circle, the others inside radius sigma)."""
    xa, pxa = _d(xa)
    ya, pya = _d(ya)
    gx, pgx = _d(gx)
    gy, pgy = _d(gy)
    tx = np.empty(xa.size)
    ty = np.empty(xa.size)
    cons = np.empty(xa.size, dtype=np.int32)
    if pin is None:
        m = lib().orc_reduce_grad(xa.size, pxa, pya, pgx, pgy, tx.ctypes.data_as(_D),
                                  ty.ctypes.data_as(_D), cons.ctypes.data_as(_I32))
    else:
        pin, ppin = _i(pin)
        m = lib().orc_reduce_grad_bi(xa.size, pxa, pya, pgx, pgy, ppin, float(sigma), tx.ctypes.data_as(_D),
                                     ty.ctypes.data_as(_D), cons.ctypes.data_as(_I32))
    return tx, ty, cons, m


def patches(x, y, centres, sizes):
    """Patch p = the sizes[p] charges nearest to charge centres[p]: squared
    distance (dx*dx)+(dy*dy) in FP64 (no fused multiply-add), ties to the lower
    index; each patch listed in increasing index order, patches concatenated."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    idx = np.arange(x.size)
    out = []
    for c, k in zip(np.asarray(centres), np.asarray(sizes)):
        dx = x - x[c]
        dy = y - y[c]
        d2 = dx * dx + dy * dy
        out.append(np.sort(np.lexsort((idx, d2))[:k]))
    return np.concatenate(out).astype(np.int32)


def spacing(n: int) -> float:
    """Mean triangular-lattice spacing for n charges in the unit disk."""
    return float(np.sqrt(2.0 * np.pi / (np.sqrt(3.0) * n)))


def relax(x, y, idx, xa=None, ya=None, gtol=1e-10, max_iter=5000, lbfgs_m=8,
          newton_tol=None, step0=None, cg_max=200, pin=None, sigma: float = 1.0):
    """Local relaxation of the active set (Sec. II.C step 4, Cartesian reading).
    pin (flags per active) and sigma select the border-interior constraint of
    Sec. II.B instead of the hard wall.

    Returns (xa, ya, stats dict)."""
    x, px = _d(x)
    y, py = _d(y)
    idx, pidx = _i(idx)
    if xa is None:
        xa = x[idx].copy()
        ya = y[idx].copy()
    xa = np.array(xa, dtype=np.float64, copy=True)
    ya = np.array(ya, dtype=np.float64, copy=True)
    h = spacing(x.size)
    o = RelaxOpts(int(max_iter), int(lbfgs_m), float(gtol),
                  float(newton_tol if newton_tol is not None else 1e-3 / h ** 2),
                  float(step0 if step0 is not None else 0.05 * h), int(cg_max))
    st = RelaxStats()
    if pin is None:
        lib().orc_relax(x.size, px, py, idx.size, pidx, xa.ctypes.data_as(_D), ya.ctypes.data_as(_D),
                        ctypes.byref(o), ctypes.byref(st))
    else:
        pin, ppin = _i(pin)
        lib().orc_relax_bi(x.size, px, py, idx.size, pidx, ppin, float(sigma), xa.ctypes.data_as(_D),
                           ya.ctypes.data_as(_D), ctypes.byref(o), ctypes.byref(st))
    return xa, ya, {"iters": st.iters, "newton_steps": st.newton_steps,
                    "status": st.status, "gtan_inf": st.gtan_inf}


def tangent_hessian_dense(x, y, idx=None, xa=None, ya=None):
    """Hessian of E_sub on the feasible tangent space at (xa, ya).

    Free charges keep both Cartesian directions; a charge held by the wall
    keeps only its tangent t = (-y, x)/|r| and gains the circle's curvature
    term -(g . r_hat).  Returns (Hr, Q) with Hr = Q^T H Q + W in the reduced
    basis Q (2na x k).  Built from the dense Hessian, so tiny sizes only."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.size
    if idx is None:
        idx = np.arange(n, dtype=np.int32)
    idx = np.asarray(idx, dtype=np.int32)
    X = x.copy()
    Y = y.copy()
    if xa is not None:
        X[idx] = xa
        Y[idx] = ya
    H = hessian(X, Y)
    sel = np.empty(2 * idx.size, dtype=np.int64)
    sel[0::2] = 2 * idx
    sel[1::2] = 2 * idx + 1
    Ha = H[np.ix_(sel, sel)]
    _, gx, gy = esub(x, y, idx, X[idx], Y[idx], grad=True)
    _, _, cons, _ = reduce_grad(X[idx], Y[idx], gx, gy)
    cols = []
    wdiag = []
    for a in range(idx.size):
        if cons[a]:
            r = np.hypot(X[idx[a]], Y[idx[a]])
            ux, uy = X[idx[a]] / r, Y[idx[a]] / r
            q = np.zeros(2 * idx.size)
            q[2 * a] = -uy
            q[2 * a + 1] = ux
            cols.append(q)
            wdiag.append(-(gx[a] * ux + gy[a] * uy))
        else:
            for c in range(2):
                q = np.zeros(2 * idx.size)
                q[2 * a + c] = 1.0
                cols.append(q)
                wdiag.append(0.0)
    Q = np.array(cols).T
    Hr = Q.T @ Ha @ Q + np.diag(wdiag)
    return 0.5 * (Hr + Hr.T), Q


def tu_grad(kind, sigma, c, gx, gy):
    """Gradient in the coordinates of Sec. II.D (kind 0 (x, y), 1 boundary
    angle, 2 interior (t, u); c interleaved per charge) from the Cartesian
    gradient, by Eqs. 8-10."""
    kind, pk = _i(kind)
    c, pc = _d(c)
    gx, pgx = _d(gx)
    gy, pgy = _d(gy)
    out = np.empty(2 * kind.size)
    lib().orc_tu_grad(kind.size, pk, float(sigma), pc, pgx, pgy, out.ctypes.data_as(_D))
    return out


def relax_tu(x, y, idx, xa=None, ya=None, pin=None, sigma: float = 1.0, gtol=1e-6, max_iter=20000,
             lbfgs_m=16, step0=None):
    """Relaxation in the (t, u) coordinates of Sec. II.D (L-BFGS; see
    oracle.c).  pin (flags per active) marks boundary charges.  Returns
    (xa, ya, stats dict)."""
    x, px = _d(x)
    y, py = _d(y)
    idx, pidx = _i(idx)
    if xa is None:
        xa = x[idx].copy()
        ya = y[idx].copy()
    xa = np.array(xa, dtype=np.float64, copy=True)
    ya = np.array(ya, dtype=np.float64, copy=True)
    if pin is None:
        pin = np.zeros(idx.size, dtype=np.int32)
    pin, ppin = _i(pin)
    h = spacing(x.size)
    o = RelaxOpts(int(max_iter), int(lbfgs_m), float(gtol), 0.0,
                  float(step0 if step0 is not None else 0.1 * h), 0)
    st = RelaxStats()
    lib().orc_relax_tu(x.size, px, py, idx.size, pidx, ppin, float(sigma), xa.ctypes.data_as(_D),
                       ya.ctypes.data_as(_D), ctypes.byref(o), ctypes.byref(st))
    return xa, ya, {"iters": st.iters, "status": st.status, "gtan_inf": st.gtan_inf}
