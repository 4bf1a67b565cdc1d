"""Perturb-and-relax cycles over random subdomains (batched candidates,
greedy commit), the driver loop of the benchmark's energy-versus-time run.

Each cycle: draw patch centres and sizes (seeded), build the patches
(k nearest charges), kick their actives with Gaussian displacements, relax
all candidates in one batched call against the current configuration, and
commit the improving ones greedily with exact energy changes re-evaluated
against the configuration as it changes.  The tracked energy (start energy
plus committed changes) is compared with a from-scratch FP64 evaluation every
cycle.  All arithmetic runs in the library; this module only sequences calls
and draws the random inputs.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import FP64, MIXED, ops, relax as R, workloads as W


def perturb_relax_cycles(x, y, cycles: int, n_patches: int = 64, size_lo: int = 200,
                         size_hi: int = 5000, kick: float = 0.3, seed: int = 1005,
                         precision: int = MIXED, gtol: float = 1e-3, log=None):
    """x, y: device float64 tensors, updated in place.  Returns a list of
    per-cycle records (cycle, wall_s, energy, tracked_energy, accepted, sum_dE)."""
    n = x.numel()
    h = W.spacing(n)
    torch.cuda.synchronize()
    E = ops.energy(x, y, FP64).item()
    tracked = E
    out = []
    t0 = time.perf_counter()
    for c in range(cycles):
        centres, sizes = W.patch_draws(n, n_patches, size_lo, size_hi, seed + 7919 * c)
        ptr, idx = R.build_patches(x, y, centres, sizes)
        kx, ky = W.kicks(int(ptr[-1]), kick * h, seed + 104729 + 7919 * c)
        idx_h = idx.cpu().numpy()
        sx, sy = W.kicked_starts(x.cpu().numpy(), y.cpu().numpy(), idx_h, kx, ky)
        dev = x.device
        res = R.relax_subdomains(x, y, ptr, idx, torch.tensor(sx, device=dev), torch.tensor(sy, device=dev),
                                 precision=precision, gtol=gtol)
        com, dc = R.commit_patches(x, y, ptr, idx, res.x, res.y, res.dE.cpu().numpy())
        tracked += float(dc[com == 1].sum())
        E = ops.energy(x, y, FP64).item()
        rec = {"cycle": c + 1, "wall_s": time.perf_counter() - t0, "energy": E, "tracked_energy": tracked,
               "accepted": int(com.sum()), "sum_dE": float(dc[com == 1].sum()),
               "relax_status": np.bincount(res.status.cpu().numpy(), minlength=4).tolist()}
        out.append(rec)
        if log is not None:
            log(rec)
    return out
