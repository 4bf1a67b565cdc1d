"""ctypes binding of the border-interior entry points (border_count,
border_sigma0, border_split): argument marshalling only.

Sec. II.B splits the charges into N_b boundary charges pinned to the unit
circle and interior charges confined to |r| <= sigma, sigma rising from the
value of Eq. 5 to 1; relax_subdomains takes the flags and sigma.
"""
from __future__ import annotations

import ctypes

import torch

from . import ops


def _lib():
    L = ops.lib()
    if not getattr(L, "_border_bound", False):
        L.border_count.restype = ctypes.c_int32
        L.border_count.argtypes = [ctypes.c_int64]
        L.border_sigma0.restype = ctypes.c_double
        L.border_sigma0.argtypes = [ctypes.c_int64]
        L.border_sigma_ramp.restype = ctypes.c_double
        L.border_sigma_ramp.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_double]
        L.border_split.restype = ctypes.c_int
        L.border_split.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p]
        L.border_project.restype = ctypes.c_int
        L.border_project.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_double, ctypes.c_void_p]
        L.border_spread.restype = ctypes.c_int
        L.border_spread.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L._border_bound = True
    return L


def boundary_count(n: int) -> int:
    """N_b of Eq. 4 (nearest integer)."""
    return int(_lib().border_count(int(n)))


def sigma0(n: int) -> float:
    """Initial interior radius of Eq. 5."""
    return float(_lib().border_sigma0(int(n)))


def sigma_ramp(k: int, stages: int, n: int, sigma_start: float = 0.0, sigma_end: float = 1.0) -> float:
    """Interior radius of stage k = 0..stages, linear from sigma_start (Eq. 5's
    value when 0) to sigma_end."""
    return float(_lib().border_sigma_ramp(int(n), int(k), int(stages), float(sigma_start), float(sigma_end)))


def border_split(x, y, nb: int):
    """Device int32 flags: 1 for the nb charges farthest from the centre."""
    dev = ops._chk(x, y)
    n = x.numel()
    flags = torch.empty(n, dtype=torch.int32, device=dev)
    ops.check(_lib().border_split(x.data_ptr(), y.data_ptr(), n, int(nb), flags.data_ptr(),
                                  ops.stream_ptr(dev)), "border_split")
    return flags


def border_project(x, y, flags, sigma: float) -> None:
    """Project (x, y) in place: flagged charges onto the unit circle, the
    others into radius sigma."""
    dev = ops._chk(x, y)
    if flags is not None and (flags.dtype != torch.int32 or flags.numel() != x.numel() or flags.device != dev):
        raise ops.CoulombError("flags must be a device int32 tensor of length n")
    ops.check(_lib().border_project(x.data_ptr(), y.data_ptr(), x.numel(),
                                    flags.data_ptr() if flags is not None else None, float(sigma),
                                    ops.stream_ptr(dev)), "border_project")


def border_spread(x, y, flags) -> None:
    """In place: the flagged charges onto the unit circle, evenly spaced in
    angle in their angular order (the split's start before a cycle)."""
    dev = ops._chk(x, y)
    if flags.dtype != torch.int32 or flags.numel() != x.numel() or flags.device != dev:
        raise ops.CoulombError("flags must be a device int32 tensor of length n")
    n = x.numel()
    ws, nb = ops.workspace(ops.OP_BORDER, n, ops.FP64, dev)
    ops.check(_lib().border_spread(x.data_ptr(), y.data_ptr(), n, flags.data_ptr(), ws.data_ptr(), nb,
                                   ops.stream_ptr(dev)), "border_spread")
