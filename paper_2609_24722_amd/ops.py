"""ctypes binding of libcoulombdisk.so: argument marshalling only.

Every function takes torch tensors that live on a GPU (float64, contiguous,
same device), sizes the library's scratch from ``coulomb_workspace_bytes``,
and enqueues on torch's current stream.  No computation happens here; if the
shared library is missing the first call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

from . import FP64, MIXED

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcoulombdisk.so")

(OP_ENERGY, OP_FORCES, OP_HVP, OP_VALIDATE, OP_PATCHES, OP_RELAX, OP_LANCZOS, OP_DEFECT, OP_ZONES,
 OP_VORONOI, OP_BORDER) = range(11)

_lib = None
_ws = {}    # (device, op, stream) -> [buffer, used under capture]
_kept = []  # outgrown buffers that a captured graph may still use

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t


class CoulombError(RuntimeError):
    pass


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CoulombError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.coulomb_workspace_bytes.restype = _sz
        L.coulomb_workspace_bytes.argtypes = [ctypes.c_int, _i64, _i32, _i64, ctypes.c_int]
        L.coulomb_energy.restype = ctypes.c_int
        L.coulomb_energy.argtypes = [_vp, _vp, _i64, ctypes.c_int, _vp, _vp, _vp, _sz, _vp]
        L.coulomb_forces.restype = ctypes.c_int
        L.coulomb_forces.argtypes = [_vp, _vp, _i64, ctypes.c_int, _vp, _vp, _vp, _vp, _sz, _vp]
        L.coulomb_hvp.restype = ctypes.c_int
        L.coulomb_hvp.argtypes = [_vp, _vp, _vp, _vp, _i64, ctypes.c_int, _vp, _vp, _vp, _sz, _vp]
        L.coulomb_validate.restype = ctypes.c_int
        L.coulomb_validate.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp, _sz, _vp]
        L.coulomb_status_string.restype = ctypes.c_char_p
        L.coulomb_status_string.argtypes = [ctypes.c_int]
        _bind_relax(L)
        _lib = L
    return _lib


def _bind_relax(L):
    if hasattr(L, "relax_subdomains"):
        from . import relax as _r  # noqa: F401  (binds its own symbols)
        _r._bind(L)


def check(rc: int, what: str) -> None:
    if rc != 0:
        raise CoulombError(f"{what}: {lib().coulomb_status_string(rc).decode()} ({rc})")


def workspace(op: int, n: int, precision: int, device, n_patches: int = 0, total_active: int = 0):
    """Device scratch for ``op`` on the current stream: grown on demand and
    cached per device, op and stream, so calls on different streams never
    share one.  A buffer that a graph capture has used is never released: when
    a later call outgrows it, the old buffer stays alive (the captured graph
    keeps writing to it on every replay) and the call gets a new one."""
    nbytes = int(lib().coulomb_workspace_bytes(op, n, n_patches, total_active, precision))
    if nbytes == 0:
        raise CoulombError(f"invalid sizes for op {op}: n={n}")
    stream = torch.cuda.current_stream(device)
    key = (str(device), op, stream.cuda_stream)
    ent = _ws.get(key)
    if ent is None or ent[0].numel() < nbytes:
        if ent is not None and ent[1]:
            _kept.append(ent[0])
        ent = [torch.empty(nbytes, dtype=torch.uint8, device=device), False]
        _ws[key] = ent
    if torch.cuda.is_current_stream_capturing():
        ent[1] = True
    return ent[0], nbytes


def stream_ptr(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _chk(*ts):
    dev = ts[0].device
    if dev.type != "cuda":
        raise CoulombError("tensors must live on a GPU")
    for t in ts:
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device != dev:
            raise CoulombError("expected contiguous float64 tensors on one device")
        if t.numel() != ts[0].numel():
            raise CoulombError("length mismatch")
    return dev


def energy(x, y, precision: int = MIXED, local: bool = False):
    """E = sum_{i<j} 1/r_ij (Eq. 2) as a 1-element tensor; with local=True
    also e_i = 1/2 sum_{j!=i} 1/r_ij (Sec. II.C step 1)."""
    dev = _chk(x, y)
    n = x.numel()
    E = torch.empty(1, dtype=torch.float64, device=dev)
    e = torch.empty(n, dtype=torch.float64, device=dev) if local else None
    ws, nb = workspace(OP_ENERGY, n, precision, dev)
    check(lib().coulomb_energy(x.data_ptr(), y.data_ptr(), n, precision, E.data_ptr(),
                               e.data_ptr() if local else None, ws.data_ptr(), nb, stream_ptr(dev)),
          "coulomb_energy")
    return (E, e) if local else E


def forces(x, y, precision: int = MIXED, with_energy: bool = True):
    """F_i = -dE/dr_i; returns (fx, fy, E or None)."""
    dev = _chk(x, y)
    n = x.numel()
    fx = torch.empty(n, dtype=torch.float64, device=dev)
    fy = torch.empty(n, dtype=torch.float64, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev) if with_energy else None
    ws, nb = workspace(OP_FORCES, n, precision, dev)
    check(lib().coulomb_forces(x.data_ptr(), y.data_ptr(), n, precision, fx.data_ptr(), fy.data_ptr(),
                               E.data_ptr() if with_energy else None, ws.data_ptr(), nb,
                               stream_ptr(dev)), "coulomb_forces")
    return fx, fy, E


def riesz(x, y, s: float, precision: int = MIXED, with_energy: bool = True):
    """Riesz-s energy sum_{i<j} r^-s and forces F_i = sum_j s (r_i - r_j) r^(-s-2);
    returns (fx, fy, E or None)."""
    dev = _chk(x, y)
    n = x.numel()
    L = lib()
    if not getattr(L, "_riesz_bound", False):
        L.coulomb_riesz.restype = ctypes.c_int
        L.coulomb_riesz.argtypes = [_vp, _vp, _i64, ctypes.c_double, ctypes.c_int, _vp, _vp, _vp, _vp, _sz, _vp]
        L._riesz_bound = True
    fx = torch.empty(n, dtype=torch.float64, device=dev)
    fy = torch.empty(n, dtype=torch.float64, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev) if with_energy else None
    ws, nb = workspace(OP_FORCES, n, precision, dev)
    check(L.coulomb_riesz(x.data_ptr(), y.data_ptr(), n, float(s), precision, fx.data_ptr(), fy.data_ptr(),
                          E.data_ptr() if with_energy else None, ws.data_ptr(), nb, stream_ptr(dev)),
          "coulomb_riesz")
    return fx, fy, E


def hvp(x, y, vx, vy, precision: int = MIXED):
    """(H v)_i = sum_{j!=i} K(d_ij)(v_i - v_j); returns (hx, hy)."""
    dev = _chk(x, y, vx, vy)
    n = x.numel()
    hx = torch.empty(n, dtype=torch.float64, device=dev)
    hy = torch.empty(n, dtype=torch.float64, device=dev)
    ws, nb = workspace(OP_HVP, n, precision, dev)
    check(lib().coulomb_hvp(x.data_ptr(), y.data_ptr(), vx.data_ptr(), vy.data_ptr(), n, precision,
                            hx.data_ptr(), hy.data_ptr(), ws.data_ptr(), nb, stream_ptr(dev)),
          "coulomb_hvp")
    return hx, hy


def autotune(x, y, op: int = OP_FORCES):
    """Time the mixed pair pass's launch shapes for `op` (OP_ENERGY,
    OP_FORCES or OP_HVP) on these positions and keep the fastest for later
    calls with the same op and n on this device.  Returns (index, waves,
    offsets per chunk)."""
    dev = _chk(x, y)
    n = x.numel()
    L = lib()
    if not getattr(L, "_tune_bound", False):
        L.coulomb_autotune.restype = ctypes.c_int
        L.coulomb_autotune.argtypes = [_vp, _vp, _i64, ctypes.c_int, _vp, _sz, _vp, _vp]
        L._tune_bound = True
    nb = int(L.coulomb_workspace_bytes(op, n, 0, 0, MIXED))
    if nb == 0:
        raise CoulombError(f"invalid sizes for op {op}: n={n}")
    nb += 16 * n + 512
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    out = (ctypes.c_int32 * 3)()
    check(L.coulomb_autotune(x.data_ptr(), y.data_ptr(), n, int(op), ws.data_ptr(), nb, stream_ptr(dev),
                             ctypes.cast(out, _vp)), "coulomb_autotune")
    return int(out[0]), int(out[1]), int(out[2])


def validate(x, y):
    """Per-charge domain flags (CD_FLAG_* bits) and the flagged count."""
    dev = _chk(x, y)
    n = x.numel()
    flags = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    ws, nb = workspace(OP_VALIDATE, n, FP64, dev)
    check(lib().coulomb_validate(x.data_ptr(), y.data_ptr(), n, flags.data_ptr(), cnt.data_ptr(),
                                 ws.data_ptr(), nb, stream_ptr(dev)), "coulomb_validate")
    return flags, cnt


def tangent_lanczos(x, y, k: int = 200, mask=None, deflate_rotation: bool = True, seed: int = 12345):
    """Smallest and largest Ritz values of the tangent-space Hessian (hard
    wall of Eq. 3) after k Lanczos steps, with the residual of the smallest.
    Returns dict(theta_min, resid, theta_max, steps, certified)."""
    dev = _chk(x, y)
    n = x.numel()
    if mask is not None and (mask.dtype != torch.int32 or mask.numel() != n or mask.device != dev):
        raise CoulombError("mask must be a device int32 tensor of length n")
    L = lib()
    if not getattr(L, "_lz_bound", False):
        L.tangent_lanczos.restype = ctypes.c_int
        L.tangent_lanczos.argtypes = [_vp, _vp, _i64, _vp, _i32, _i32, ctypes.c_uint64, _vp, _vp, _sz, _vp]
        L._lz_bound = True
    ws, nb = workspace(OP_LANCZOS, n, FP64, dev, n_patches=int(k))
    out = (ctypes.c_double * 4)()
    check(L.tangent_lanczos(x.data_ptr(), y.data_ptr(), n, mask.data_ptr() if mask is not None else None,
                            int(k), int(bool(deflate_rotation)), int(seed), ctypes.cast(out, _vp),
                            ws.data_ptr(), nb, stream_ptr(dev)), "tangent_lanczos")
    th, res, tmax, steps = out[0], out[1], out[2], int(out[3])
    return {"theta_min": th, "resid": res, "theta_max": tmax, "steps": steps,
            "certified": bool(th > 0 and res < 0.5 * th)}
