"""ctypes binding of the zone entry points (defect_zones, zone_patches,
zone_batches): argument marshalling only.

Zones are the subdomains of the paper's defect-targeted cycle (Sec. II.C):
a centre (a defect charge or a uniform point of the disk), a radius that
oscillates over the cycle, and every charge within that radius.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import ops

_vp = ctypes.c_void_p
CD_ERR_CAPACITY = -5


class ZoneOpts(ctypes.Structure):
    _fields_ = [
        ("kappa", ctypes.c_double),
        ("p_defect", ctypes.c_double),
        ("r_lo", ctypes.c_double),
        ("r_hi", ctypes.c_double),
        ("t0", ctypes.c_int64),
        ("period", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


def _lib():
    L = ops.lib()
    if not getattr(L, "_zones_bound", False):
        L.defect_zones.restype = ctypes.c_int
        L.defect_zones.argtypes = [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp,
                                   ctypes.POINTER(ZoneOpts), _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   ctypes.c_size_t, _vp]
        L.zone_patches.restype = ctypes.c_int
        L.zone_patches.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp,
                                   ctypes.c_int64, _vp, ctypes.c_size_t, _vp]
        L.zone_batches.restype = ctypes.c_int
        L.zone_batches.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                   ctypes.c_int32, _vp, _vp]
        L.zone_radius_holding.restype = ctypes.c_double
        L.zone_radius_holding.argtypes = [ctypes.c_int64, ctypes.c_int64]
        L._zones_bound = True
    return L


def radius_holding(n: int, count: int) -> float:
    """Radius of a disk that holds `count` of n charges at the mean density."""
    return float(_lib().zone_radius_holding(int(n), int(count)))


def defect_zones(x, y, e, draws, kappa: float = -1.0, p_defect: float = 0.8, r_lo: float = 0.0,
                 r_hi: float = 0.0, t0: int = 0, period: int = 1):
    """Steps 2-3 of Sec. II.C from the local energies e (device float64 [n])
    and the draws (device float64 [4 P]: u, v, px, py per zone).  Returns a
    dict of device tensors: cx, cy, rz [P], centre_idx [P] (-1 for a disk
    point), stats [4] (mu, sigma_e, threshold, defect count) and defects
    [n] (its first `count` entries are the defect list)."""
    dev = ops._chk(x, y, e)
    n = x.numel()
    if draws.dtype != torch.float64 or draws.device != dev or not draws.is_contiguous() or draws.numel() % 4:
        raise ops.CoulombError("draws must be a contiguous device float64 tensor of 4 values per zone")
    P = draws.numel() // 4
    f = dict(dtype=torch.float64, device=dev)
    cx, cy, rz = torch.empty(P, **f), torch.empty(P, **f), torch.empty(P, **f)
    ci = torch.empty(P, dtype=torch.int32, device=dev)
    stats = torch.empty(4, **f)
    defects = torch.empty(n, dtype=torch.int32, device=dev)
    o = ZoneOpts(float(kappa), float(p_defect), float(r_lo), float(r_hi), int(t0), int(period), 0)
    ws, nb = ops.workspace(ops.OP_DEFECT, n, ops.FP64, dev)
    ops.check(_lib().defect_zones(x.data_ptr(), y.data_ptr(), e.data_ptr(), n, P,
                                  draws.data_ptr() if P else None, ctypes.byref(o),
                                  cx.data_ptr() if P else None, cy.data_ptr() if P else None,
                                  rz.data_ptr() if P else None, ci.data_ptr() if P else None,
                                  stats.data_ptr(), defects.data_ptr(), ws.data_ptr(), nb,
                                  ops.stream_ptr(dev)), "defect_zones")
    return {"cx": cx, "cy": cy, "rz": rz, "centre_idx": ci, "stats": stats, "defects": defects}


def zone_patches(x, y, cx, cy, rz, capacity: int = 0):
    """Every charge within rz[p] of (cx[p], cy[p]), per zone in increasing
    index order (Sec. II.C step 4).  Returns (ptr host int32 [P+1], idx
    device int32).  `capacity` is a first guess of the total; a second pass
    runs when it is too small."""
    dev = ops._chk(x, y)
    ops._chk(cx, cy, rz)
    n = x.numel()
    P = cx.numel()
    if P < 1:
        raise ops.CoulombError("no zones")
    ptr = np.zeros(P + 1, dtype=np.int32)
    ws, nb = ops.workspace(ops.OP_ZONES, n, ops.FP64, dev, n_patches=P)
    L = _lib()
    for cap in (int(capacity), None):
        if cap is None:
            cap = int(ptr[-1])
        idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        rc = L.zone_patches(x.data_ptr(), y.data_ptr(), n, P, cx.data_ptr(), cy.data_ptr(), rz.data_ptr(),
                            ptr.ctypes.data, idx.data_ptr(), cap, ws.data_ptr(), nb, ops.stream_ptr(dev))
        if rc != CD_ERR_CAPACITY:
            ops.check(rc, "zone_patches")
            return ptr, idx[:int(ptr[-1])]
    raise ops.CoulombError("zone_patches: capacity still too small")


def zone_batches(cx, cy, rz, gap: float, cap: int, keep_order: bool = False):
    """Batch index of each zone (host numpy arrays in, int32 array out) and
    the number of batches: zones of one batch are apart by more than gap;
    keep_order puts each zone after every earlier one it conflicts with,
    otherwise each goes to the first batch free of conflicts."""
    cx = np.ascontiguousarray(cx, dtype=np.float64)
    cy = np.ascontiguousarray(cy, dtype=np.float64)
    rz = np.ascontiguousarray(rz, dtype=np.float64)
    T = cx.size
    batch = np.zeros(T, dtype=np.int32)
    nb = np.zeros(1, dtype=np.int32)
    ops.check(_lib().zone_batches(cx.ctypes.data, cy.ctypes.data, rz.ctypes.data, T, float(gap), int(cap),
                                  int(bool(keep_order)), batch.ctypes.data, nb.ctypes.data), "zone_batches")
    return batch, int(nb[0])
