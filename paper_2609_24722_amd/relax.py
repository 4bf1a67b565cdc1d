"""ctypes binding of the subdomain entry points (build_patches,
relax_subdomains): argument marshalling only.

A batch of P patches is given by host offsets ``ptr`` (numpy int32, length
P+1) and a device int32 tensor of charge indices (packed per patch).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import FP64, MIXED
from . import ops

_vp = ctypes.c_void_p


class RelaxOpts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("lbfgs_m", ctypes.c_int32),
        ("max_outer", ctypes.c_int32),
        ("gtol", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
        ("halo_width", ctypes.c_double),
        ("step0", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("boundary", ctypes.c_void_p),
        ("polish", ctypes.c_int32),
        ("max_polish_iter", ctypes.c_int32),
        ("newton_tol", ctypes.c_double),
        ("cg_eta", ctypes.c_double),
        ("polish_stats", ctypes.c_void_p),
        ("trust_radius", ctypes.c_double),
        ("coords", ctypes.c_int32),
        ("launch", ctypes.c_int32),
        ("exterior_model", ctypes.c_int32),
    ]

# polish modes of relax_subdomains
POLISH_DEFAULT, POLISH_NEWTON, POLISH_LBFGS = 0, 1, 2
# coordinates of interior charges: (x, y) under the wall rule, or (t, u) of Sec. II.D
COORDS_XY, COORDS_TU = 0, 1
# lock-step rounds replayed from HIP graphs, or launched one by one
LAUNCH_GRAPH, LAUNCH_PLAIN = 0, 1
# exterior of the relax: set by precision, exact FP64 evaluations, or the halo + far-field model
EXTERIOR_DEFAULT, EXTERIOR_EXACT, EXTERIOR_MODEL = 0, 1, 2
# candidates of relax_autotune
RELAX_SCHEDULES = 9


def _bind(L):
    L.commit_patches.restype = ctypes.c_int
    L.commit_patches.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp,
                                 _vp, _vp, ctypes.c_size_t, _vp]
    L.build_patches.restype = ctypes.c_int
    L.build_patches.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, _vp,
                                ctypes.c_size_t, _vp]
    L.relax_subdomains.restype = ctypes.c_int
    L.relax_subdomains.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, _vp,
                                   ctypes.POINTER(RelaxOpts), _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                   _vp, ctypes.c_size_t, _vp]


def offsets(sizes) -> np.ndarray:
    sizes = np.asarray(sizes, dtype=np.int64)
    ptr = np.zeros(sizes.size + 1, dtype=np.int32)
    ptr[1:] = np.cumsum(sizes)
    return ptr


def build_patches(x, y, centres, sizes):
    """The sizes[p] charges nearest to charge centres[p] (Sec. II.C steps 3-4),
    per patch in increasing index order.  Returns (ptr host int32, idx device)."""
    dev = ops._chk(x, y)
    n = x.numel()
    ptr = offsets(sizes)
    c = torch.as_tensor(np.asarray(centres, dtype=np.int32), device=dev)
    idx = torch.empty(int(ptr[-1]), dtype=torch.int32, device=dev)
    ws, nb = ops.workspace(ops.OP_PATCHES, n, ops.FP64, dev, n_patches=ptr.size - 1)
    ops.check(ops.lib().build_patches(x.data_ptr(), y.data_ptr(), n, ptr.size - 1, c.data_ptr(),
                                      ptr.ctypes.data, idx.data_ptr(), ws.data_ptr(), nb,
                                      ops.stream_ptr(dev)), "build_patches")
    return ptr, idx


@dataclass
class RelaxResult:
    x: torch.Tensor        # packed relaxed positions
    y: torch.Tensor
    dE: torch.Tensor       # [P] E_sub(relaxed) - E_sub(snapshot), exact FP64
    e_sub: torch.Tensor    # [P] exact E_sub at the relaxed positions
    gtan_inf: torch.Tensor  # [P] exact reduced-gradient inf-norm
    iters: torch.Tensor    # [P, 2] accepted iterations (L-BFGS and Newton), exact evaluations
    status: torch.Tensor   # [P] 0 converged, 1 cap, 2 line search failed, 3 non-finite
    polish: torch.Tensor   # [P, 2] accepted Newton steps, CG iterations


def relax_subdomains(x, y, ptr, idx, x_start=None, y_start=None, precision=MIXED, gtol=1e-3,
                     max_iter=None, lbfgs_m=16, max_outer=0, inner_tol=0.0, halo_width=0.0,
                     step0=0.0, sigma=0.0, boundary=None, polish=POLISH_DEFAULT, max_polish_iter=0,
                     newton_tol=0.0, cg_eta=0.0, trust_radius=0.0, coords=COORDS_XY,
                     launch=LAUNCH_GRAPH, exterior_model=EXTERIOR_DEFAULT) -> RelaxResult:
    """Relax every patch against the frozen snapshot (x, y); see coulomb_disk.h.

    max_iter defaults to 300 per round for the mixed path and 8000 in total for
    the FP64 path.  boundary (device int32 [n]) and sigma select the
    border-interior split of Sec. II.B.  polish, max_polish_iter, newton_tol
    and cg_eta set the truncated-Newton polish, trust_radius (units of h) the
    mixed path's model radius (0: the library defaults); coords COORDS_TU
    moves interior charges in the (t, u) of Sec. II.D; launch picks graph
    replays or plain launches of the lock-step rounds; exterior_model
    EXTERIOR_MODEL with FP64 runs the model with FP64 pairs throughout."""
    if max_iter is None:
        max_iter = 300 if precision == MIXED else 8000
    dev = ops._chk(x, y)
    n = x.numel()
    ptr = np.ascontiguousarray(ptr, dtype=np.int32)
    P = ptr.size - 1
    ntot = int(ptr[-1])
    if idx.dtype != torch.int32 or idx.numel() != ntot or idx.device != dev:
        raise ops.CoulombError("idx must be a device int32 tensor of length ptr[-1]")
    if x_start is not None:
        ops._chk(x_start, y_start)
        if x_start.numel() != ntot:
            raise ops.CoulombError("start positions must be packed like idx")
    if boundary is not None and (boundary.dtype != torch.int32 or boundary.numel() != n
                                 or boundary.device != dev):
        raise ops.CoulombError("boundary must be a device int32 tensor of length n")
    pst = torch.empty((P, 2), dtype=torch.int32, device=dev)
    o = RelaxOpts(int(precision), int(max_iter), int(lbfgs_m), int(max_outer), float(gtol),
                  float(inner_tol), float(halo_width), float(step0), float(sigma),
                  boundary.data_ptr() if boundary is not None else None, int(polish),
                  int(max_polish_iter), float(newton_tol), float(cg_eta), pst.data_ptr(),
                  float(trust_radius), int(coords), int(launch), int(exterior_model))
    f = dict(dtype=torch.float64, device=dev)
    xo = torch.empty(ntot, **f)
    yo = torch.empty(ntot, **f)
    dE = torch.empty(P, **f)
    es = torch.empty(P, **f)
    gt = torch.empty(P, **f)
    it = torch.empty((P, 2), dtype=torch.int32, device=dev)
    stt = torch.empty(P, dtype=torch.int32, device=dev)
    ws_prec = MIXED if exterior_model == EXTERIOR_MODEL else int(precision)
    ws, nb = ops.workspace(ops.OP_RELAX, n, ws_prec, dev, n_patches=P, total_active=ntot)
    ops.check(ops.lib().relax_subdomains(
        x.data_ptr(), y.data_ptr(), n, P, ptr.ctypes.data, idx.data_ptr(),
        x_start.data_ptr() if x_start is not None else None,
        y_start.data_ptr() if y_start is not None else None, ctypes.byref(o),
        xo.data_ptr(), yo.data_ptr(), dE.data_ptr(), es.data_ptr(), gt.data_ptr(), it.data_ptr(),
        stt.data_ptr(), ws.data_ptr(), nb, ops.stream_ptr(dev)), "relax_subdomains")
    return RelaxResult(xo, yo, dE, es, gt, it, stt, pst)


def relax_autotune(x, y, ptr, idx, x_start=None, y_start=None, precision=MIXED, gtol=1e-3, max_iter=None,
                   lbfgs_m=16, sigma=0.0, boundary=None, coords=COORDS_XY):
    """Time every relax schedule on this batch and keep the fastest for later
    relax_subdomains calls with the same precision, coordinates, n and
    log2(total actives) (see coulomb_disk.h).  Returns (index, wide-block
    count, rounds per graph replay, polish flag, seconds per candidate)."""
    if max_iter is None:
        max_iter = 300 if precision == MIXED else 8000
    dev = ops._chk(x, y)
    n = x.numel()
    ptr = np.ascontiguousarray(ptr, dtype=np.int32)
    P = ptr.size - 1
    L = ops.lib()
    if not getattr(L, "_rtune_bound", False):
        L.relax_autotune.restype = ctypes.c_int
        L.relax_autotune.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, _vp,
                                     ctypes.POINTER(RelaxOpts), _vp, ctypes.c_size_t, _vp, _vp, _vp]
        L._rtune_bound = True
    o = RelaxOpts(int(precision), int(max_iter), int(lbfgs_m), 0, float(gtol), 0.0, 0.0, 0.0, float(sigma),
                  boundary.data_ptr() if boundary is not None else None, 0, 0, 0.0, 0.0, None, 0.0, int(coords),
                  LAUNCH_GRAPH, EXTERIOR_DEFAULT)
    ws, nb = ops.workspace(ops.OP_RELAX, n, int(precision), dev, n_patches=P, total_active=int(ptr[-1]))
    out = (ctypes.c_int32 * 4)()
    times = (ctypes.c_double * RELAX_SCHEDULES)()
    ops.check(L.relax_autotune(x.data_ptr(), y.data_ptr(), n, P, ptr.ctypes.data, idx.data_ptr(),
                               x_start.data_ptr() if x_start is not None else None,
                               y_start.data_ptr() if y_start is not None else None, ctypes.byref(o),
                               ws.data_ptr(), nb, ops.stream_ptr(dev), ctypes.cast(out, _vp),
                               ctypes.cast(times, _vp)), "relax_autotune")
    return int(out[0]), int(out[1]), int(out[2]), int(out[3]), list(times)


def commit_patches(x, y, ptr, idx, x_rel, y_rel, order_key):
    """Greedy commit (see coulomb_disk.h): updates x, y in place; returns
    (committed host int32 [P], dE_commit host float64 [P])."""
    dev = ops._chk(x, y)
    n = x.numel()
    ptr = np.ascontiguousarray(ptr, dtype=np.int32)
    P = ptr.size - 1
    key = np.ascontiguousarray(order_key, dtype=np.float64)
    com = np.zeros(P, dtype=np.int32)
    dc = np.zeros(P, dtype=np.float64)
    maxp = int(np.max(np.diff(ptr)))
    need = int(ops.lib().coulomb_workspace_bytes(ops.OP_RELAX, n, 1, maxp, FP64)) + 512
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    ops.check(ops.lib().commit_patches(x.data_ptr(), y.data_ptr(), n, P, ptr.ctypes.data, idx.data_ptr(),
                                       x_rel.data_ptr(), y_rel.data_ptr(), key.ctypes.data, com.ctypes.data,
                                       dc.ctypes.data, ws.data_ptr(), need, ops.stream_ptr(dev)),
              "commit_patches")
    return com, dc
