"""ctypes binding of the structure-analysis entry points
(voronoi_coordination, radial_histogram): argument marshalling only.

Sec. III analyses the relaxed configurations by Voronoi coordination (the
fraction of sixfold cells), the bond-orientational order psi_6 and the radial
density profile.
"""
from __future__ import annotations

import ctypes

import torch

from . import ops

_vp = ctypes.c_void_p


def _lib():
    L = ops.lib()
    if not getattr(L, "_structure_bound", False):
        L.voronoi_coordination.restype = ctypes.c_int
        L.voronoi_coordination.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp, ctypes.c_size_t, _vp]
        L.radial_histogram.restype = ctypes.c_int
        L.radial_histogram.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp]
        L.structure_stats.restype = ctypes.c_int
        L.structure_stats.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp]
        L._structure_bound = True
    return L


def voronoi(x, y, with_psi6: bool = True):
    """(z device int32 [n], psi6 device complex128 [n] or None); z = -2 marks a
    charge on the convex hull (unbounded cell)."""
    dev = ops._chk(x, y)
    n = x.numel()
    z = torch.empty(n, dtype=torch.int32, device=dev)
    psi = torch.empty(2 * n, dtype=torch.float64, device=dev) if with_psi6 else None
    ws, nb = ops.workspace(ops.OP_VORONOI, n, ops.FP64, dev)
    ops.check(_lib().voronoi_coordination(x.data_ptr(), y.data_ptr(), n, z.data_ptr(),
                                          psi.data_ptr() if with_psi6 else None, ws.data_ptr(), nb,
                                          ops.stream_ptr(dev)), "voronoi_coordination")
    return z, (torch.view_as_complex(psi.view(n, 2)) if with_psi6 else None)


def radial_histogram(x, y, nbins: int):
    dev = ops._chk(x, y)
    counts = torch.empty(int(nbins), dtype=torch.int32, device=dev)
    ops.check(_lib().radial_histogram(x.data_ptr(), y.data_ptr(), x.numel(), int(nbins), counts.data_ptr(),
                                      ops.stream_ptr(dev)), "radial_histogram")
    return counts


def stats(z, psi=None):
    """Host dict of structure_stats over a voronoi() result: P(z) for z = 4..8
    and mean |psi_6| over the bounded cells, and the cell counts."""
    dev = z.device
    if z.dtype != torch.int32 or not z.is_contiguous() or dev.type != "cuda":
        raise ops.CoulombError("z must be a contiguous device int32 tensor")
    n = z.numel()
    p = None
    if psi is not None:
        p = torch.view_as_real(psi).contiguous()
        if p.dtype != torch.float64 or p.numel() != 2 * n or p.device != dev:
            raise ops.CoulombError("psi must be a device complex128 tensor of length n")
    out = torch.empty(9, dtype=torch.float64, device=dev)
    ops.check(_lib().structure_stats(z.data_ptr(), p.data_ptr() if p is not None else None, n, out.data_ptr(),
                                     ops.stream_ptr(dev)), "structure_stats")
    o = out.cpu().tolist()
    return {"P_z": {k: o[k - 4] for k in (4, 5, 6, 7, 8)}, "mean_abs_psi6": o[5], "bounded_cells": int(o[6]),
            "hull": int(o[7]), "unresolved": int(o[8])}


def summary(x, y, nbins: int = 50):
    """Coordination fractions, <|psi_6|>, unresolved cells and radial counts
    (host values) of a configuration."""
    z, psi = voronoi(x, y)
    c = radial_histogram(x, y, nbins)
    st = stats(z, psi)
    return {"n": x.numel(), "bounded_cells": st["bounded_cells"], "hull": st["hull"],
            "unresolved": st["unresolved"], "P_z": st["P_z"], "mean_abs_psi6": st["mean_abs_psi6"],
            "radial_counts": c.cpu().tolist()}
